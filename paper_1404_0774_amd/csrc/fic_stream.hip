// fic_stream.hip -- the code stream: the codes of an encode written as a
// compact bit stream (Section IV saves the codes to the encoding file; Table
// III reports the size reduction this buys) and read back.
//
// Format (the paper gives none): a 32-byte header, then one fixed-width
// record per range.  Range r occupies payload bits [r B, (r + 1) B),
// B = D + 3 + s_bits + o_bits with D the bits that index the N_d domains;
// a record holds, from its first bit, the domain index, the transform, the
// contrast index and the offset index, each least significant bit first.
// Payload bit i is bit (i mod 32) of little-endian 32-bit word i / 32, which
// is bit (i mod 8) of byte i / 8; the payload is padded with zeros to whole
// words.  Fixed-width records make both directions embarrassingly parallel:
// one thread per output word when writing, one per range when reading.
#include "fic_internal.h"

namespace fic {

namespace {

// Record of range r: the four fields, each masked to its width.
__device__ __forceinline__ unsigned long long record(const StreamGeo &sg,
                                                     const int32_t *domain,
                                                     const uint8_t *iso,
                                                     const uint8_t *s_idx,
                                                     const uint8_t *o_idx,
                                                     long long r) {
  const unsigned long long d =
      (unsigned long long)(unsigned)domain[r] & ((1ull << sg.D) - 1ull);
  const unsigned long long k = iso[r] & 7u;
  const unsigned long long j = s_idx[r] & ((1u << sg.sb) - 1u);
  const unsigned long long m = o_idx[r] & ((1u << sg.ob) - 1u);
  return d | (k << sg.D) | (j << (sg.D + 3)) | (m << (sg.D + 3 + sg.sb));
}

// One thread per payload word (and the header from the first eight threads
// of the last workgroup).
__global__ __launch_bounds__(256) void k_stream_pack(
    StreamGeo sg, const int32_t *domain, const uint8_t *iso,
    const uint8_t *s_idx, const uint8_t *o_idx, uint32_t *out) {
  const long long w = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (w < sg.words) {
    const long long wb = 32ll * w;
    const long long r0 = wb / sg.B;
    const long long r1 = min((wb + 31) / sg.B, sg.R - 1);
    uint32_t acc = 0;
    for (long long r = r0; r <= r1; ++r) {
      const long long rs = r * sg.B;
      const unsigned long long v = record(sg, domain, iso, s_idx, o_idx, r);
      acc |= rs >= wb ? (uint32_t)(v << (rs - wb)) : (uint32_t)(v >> (wb - rs));
    }
    out[8 + w] = acc;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x < 8)
    out[threadIdx.x] = sg.header[threadIdx.x];
}

// One thread per range: the record starting at bit r B spans at most three
// payload words (B <= 64, offset within the first word <= 31).
__global__ __launch_bounds__(256) void k_stream_unpack(
    StreamGeo sg, const uint32_t *in, int32_t *domain, uint8_t *iso,
    uint8_t *s_idx, uint8_t *o_idx) {
  const long long r = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= sg.R) return;
  const long long rs = r * sg.B;
  const long long wi = rs / 32;
  const int sh = (int)(rs % 32);
  const uint32_t *pay = in + 8;
  const unsigned long long w0 = pay[wi];
  const unsigned long long w1 = wi + 1 < sg.words ? pay[wi + 1] : 0u;
  const unsigned long long w2 = wi + 2 < sg.words ? pay[wi + 2] : 0u;
  unsigned long long v = (w0 | (w1 << 32)) >> sh;
  if (sh) v |= w2 << (64 - sh);
  domain[r] = (int32_t)(v & ((1ull << sg.D) - 1ull));
  iso[r] = (uint8_t)((v >> sg.D) & 7u);
  s_idx[r] = (uint8_t)((v >> (sg.D + 3)) & ((1u << sg.sb) - 1u));
  o_idx[r] = (uint8_t)((v >> (sg.D + 3 + sg.sb)) & ((1u << sg.ob) - 1u));
}

}  // namespace

hipError_t launch_stream_pack(const StreamGeo &sg, const int32_t *domain,
                              const uint8_t *iso, const uint8_t *s_idx,
                              const uint8_t *o_idx, void *out,
                              hipStream_t st) {
  const long long blocks = (sg.words + 255) / 256;
  hipLaunchKernelGGL(k_stream_pack, dim3((unsigned)(blocks > 0 ? blocks : 1)),
                     dim3(256), 0, st, sg, domain, iso, s_idx, o_idx,
                     (uint32_t *)out);
  return hipGetLastError();
}

hipError_t launch_stream_unpack(const StreamGeo &sg, const void *in,
                                int32_t *domain, uint8_t *iso, uint8_t *s_idx,
                                uint8_t *o_idx, hipStream_t st) {
  const long long blocks = (sg.R + 255) / 256;
  hipLaunchKernelGGL(k_stream_unpack, dim3((unsigned)blocks), dim3(256), 0, st,
                     sg, (const uint32_t *)in, domain, iso, s_idx, o_idx);
  return hipGetLastError();
}

}  // namespace fic

"""Fractal (PIFS) image encoding on AMD Instinct MI355X.

The compute path lives in libfic.so (hand-written HIP for gfx950, built by
``paper_1404_0774_amd.build``); this package only marshals arguments to its C
ABI.  PyTorch provides device memory and streams.
"""
from ._lib import (FicError, Params, encode, decode, decode_batch, decode_scaled, decode_backward,
                   decode_backward_batch,
                   query,
                   dequantize, FicDecode, lib, METHOD_MFMA, METHOD_DIRECT,
                   METHOD_MFMA_I8,
                   timing_begin, timing_end, refine, Batch, Tuning, set_tuning,
                   load_tuning, get_tuning, search_counts, stream_query,
                   stream_pack, stream_header, stream_unpack, quadtree_query,
                   encode_quadtree)

__all__ = ["FicError", "Params", "encode", "decode", "decode_batch", "decode_scaled", "decode_backward",
           "decode_backward_batch",
           "query",
           "dequantize", "FicDecode", "lib", "METHOD_MFMA", "METHOD_DIRECT",
           "METHOD_MFMA_I8",
           "timing_begin", "timing_end", "refine", "Batch", "Tuning", "set_tuning",
           "load_tuning", "get_tuning", "search_counts", "stream_query",
           "stream_pack", "stream_header", "stream_unpack", "quadtree_query",
           "encode_quadtree"]

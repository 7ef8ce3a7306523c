"""The launch-shape autotuner on one point of each sweep: it times the
shape, checks that the codes do not change, and its entries load back into
the library's table and resolve for the workload they were made for."""
import json

import numpy as np
import pytest
import torch

import paper_1404_0774_amd as F
from paper_1404_0774_amd import autotune as A
from fic_inputs import gen_image

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def restore_table():
    yield
    F.set_tuning([])
    F.load_tuning(F._lib.TUNING_PATH)


def test_one_point_single_and_batch_sweep(tmp_path):
    dev = torch.device("cuda:0")
    logs = []
    img = torch.from_numpy(gen_image(128, 128, 8, 61)).to(dev)
    p = F.Params(128, 128, 8, 8, 4)
    entry, rec = A.tune_single("u8_128", img, p, [3], [0], 3, dev, logs.append)
    assert (entry["col_chunks"], entry["seed_blocks"]) == (3, 0)
    assert entry["min_domains"] == F.query(p)[1]
    assert len(rec["sweep"]) == 1 and rec["sweep"][0]["ms"] > 0 and rec["ms_default"] > 0
    sides = [64, 96, 128]
    imgs = [torch.from_numpy(gen_image(s, s, 8, 62 + i)).to(dev) for i, s in enumerate(sides)]
    params = [F.Params(s, s, 8, 8, 8) for s in sides]
    bentry, brec = A.tune_batch(imgs, params, [2], [0], 3, dev, logs.append)
    assert (bentry["item_blocks"], bentry["seed_blocks"]) == (2, 0)
    assert len(brec["sweep"]) == 1 and len(logs) == 2
    # the entries written as the tuner writes them load back and resolve
    path = tmp_path / "tuning.json"
    path.write_text(json.dumps({"entries": [entry, bentry]}))
    F.load_tuning(str(path))
    got = F.get_tuning(p)
    assert (got["col_chunks"], got["seed_blocks"]) == (3, 0)
    ref = F.encode(img, F.Params(128, 128, 8, 8, 4))
    torch.cuda.synchronize()
    F.set_tuning([])
    base = F.encode(img, F.Params(128, 128, 8, 8, 4))
    torch.cuda.synchronize()
    for k in ("domain", "iso", "s_idx", "o_idx", "err"):
        assert np.array_equal(ref[k].cpu().numpy(), base[k].cpu().numpy())

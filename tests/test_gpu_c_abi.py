"""The whole embedding called from plain C (tests/c_abi/embed_file.c, built by
build(): include/lne.h and the HIP runtime only, default stream, hipMalloc)
returns bit for bit the embedding of the same graph and parameters through
the Python binding, with 64- and with 32-bit row offsets."""
import math
import os
import subprocess

import numpy as np
import pytest
import torch

from synth import chung_lu
from tests.conftest import to_dev

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "embed_file")


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_c_caller_matches_binding(lne, ctx, tmp_path, bits, precision):
    assert os.path.exists(EXE), "tests/c_abi/embed_file is built by __graft_entry__.build()"
    g = chung_lu(2000, 16000, 2.1, seed=5)
    p = dict(T=4, s=[0.4, 0.3, 0.2, 0.1], M=6 * 4 * g.m, b=1, C=math.log(g.n), d=12,
             oversample=6, q=2, cheb_k=5, theta=0.5, mu=0.2, seed=17, precision=precision)
    rp64 = g.rowptr.astype(np.int64)
    rp_file = rp64 if bits == 64 else rp64.astype(np.int32)
    inp = tmp_path / "graph.bin"
    with open(inp, "wb") as f:
        f.write(np.array([g.n, len(g.col)], dtype=np.int64).tobytes())
        f.write(np.array([bits, 0], dtype=np.int32).tobytes())
        f.write(bytes(lne.make_params(p)))
        f.write(rp_file.tobytes())
        f.write(g.col.astype(np.int32).tobytes())
    out = tmp_path / "x.bin"
    print("c caller", bits, precision, flush=True)
    r = subprocess.run([EXE, str(inp), str(out)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    dt = np.float64 if precision == "f64" else np.float32
    Xc = np.fromfile(out, dtype=dt).reshape(g.n, p["d"])
    rp, col = to_dev(g)
    if bits == 32:
        rp = rp.to(torch.int32)
    X, st = lne.embed(ctx, rp, col, p)
    np.testing.assert_array_equal(Xc, X.cpu().numpy())
    assert f"accepted {st['accepted']} " in r.stdout

"""Full-size workloads on the GPU, checked at sampled pad columns against expected
values the FP64 oracle wrote (tests/golden/make_samples.py), and by properties that
hold at any size (zero mean after the update, linearity, bitwise repeatability)."""
import os

import numpy as np
import pytest

import fbc_workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    p = os.path.join(HERE, "golden", f"{name}_samples.npz")
    if not os.path.exists(p):
        pytest.skip(f"no stored oracle samples for {name}")
    return np.load(p)


def _digest(f):
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(f).tobytes()).hexdigest()


def rel_err(got, ref):
    n = ref.shape[0]
    g = got.reshape(n, -1)
    r = ref.reshape(n, -1)
    return float((np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)).max())


@pytest.mark.parametrize("name,form,bound", [
    ("medium", "fp64", 1e-10), ("medium", "fp32", 1e-6), ("medium", "split_bf16", 2e-5),
    ("medium", "split_fp16", 1e-6), ("medium", "dtable_fp64", 1e-10),
    ("large", "fp64", 1e-10), ("large", "split_bf16", 2e-5), ("large", "split_fp16", 1e-6),
])
def test_fullsize_green_apply_matches_oracle_samples(name, form, bound):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = _golden(name)
    wl = W.make_single(name)
    c = wl.cells[0]
    assert str(gold["digest"]) == _digest(c.forces), "seeded forces changed since the samples were written"
    from paper_2105_08798_amd import FBC
    dev = torch.device("cuda:0")
    print(f"[{name}/{form}] assembling", flush=True)
    ctx = FBC(wl.cells, wl.bz, form=form)
    f = torch.from_numpy(c.forces).to(dev)
    w = torch.zeros((c.n_rhs, c.nz, c.n_b, 3), dtype=torch.float64, device=dev)
    ctx.green_apply(f, w)
    assert ctx.sync_status() == 0
    cols = torch.from_numpy(gold["cols"]).to(dev)
    got = w[:, :, cols, :].cpu().numpy()
    # the full update keeps zero mean over the pad per RHS and component
    u = torch.zeros_like(w)
    ctx.apply(f, u, alpha=1.0)
    assert ctx.sync_status() == 0
    mean = u.mean(dim=(1, 2)).abs().max().item()
    scale = u.abs().max().item()
    ctx.close()
    del w, u, f
    torch.cuda.empty_cache()
    e = rel_err(got, gold["w"])
    print(f"[{name}/{form}] rel err vs oracle samples {e:.3e}; |mean| {mean:.1e} of {scale:.1e}", flush=True)
    assert e < bound
    assert mean < 1e-12 * scale

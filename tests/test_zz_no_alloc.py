"""The allocation-free entry point zolo_residuals_noalloc against zolo_residuals.

Both run the same fused residual kernels; the allocation-free one keeps its
partial sums in the library's static device array, which later calls reuse.
Two calls in a row (the second on a smaller input: another pencil and fewer
columns) must give exactly the allocating entry point's norms, and a column
count above the array's limit must be rejected with ZOLO_EINVAL.
"""
import sys

import numpy as np
import pytest

import pencils

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
zolo = pytest.importorskip("paper_1701_08935_amd")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return zolo.Context(0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _case(ctx, gen, shape, p, seed):
    gp = getattr(pencils, gen)(shape[0], ny=shape[1], nz=shape[2])
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=16)
    X = _dev(pencils.gaussian_block(gp.n, p, seed=seed, complex_=gen == "grid27p"))
    lam = _dev(np.random.Generator(np.random.PCG64(seed + 1)).uniform(-3.0, 9.0, p))
    return P, X, lam


@pytest.mark.parametrize("gen", ["grid7", "grid27p"])
def test_noalloc_matches_allocating_entry_point(ctx, gen):
    big = (16, 15, 14) if gen == "grid7" else (9, 10, 8)
    small = (6, 5, 7)
    for shape, p, seed in ((big, 300, 21), (small, 17, 23)):
        say(f"residuals_noalloc {gen} {shape} p={p}")
        P, X, lam = _case(ctx, gen, shape, p, seed)
        ref = zolo.zolo_residuals(P, X, lam).cpu().numpy()
        out = torch.full((p,), float("nan"), dtype=torch.float64, device="cuda:0")
        got = zolo.zolo_residuals_noalloc(P, X, lam, out)
        torch.cuda.synchronize()
        got = got.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref), np.max(np.abs(got - ref))


def test_noalloc_rejects_too_many_columns(ctx):
    say("residuals_noalloc column limit")
    P, X, lam = _case(ctx, "grid7", (4, 4, 4), 513, 31)
    out = torch.zeros(513, dtype=torch.float64, device="cuda:0")
    with pytest.raises(zolo.ZoloError) as ei:
        zolo.zolo_residuals_noalloc(P, X, lam, out)
    assert ei.value.status == zolo.ZOLO_EINVAL
    assert "limit" in str(ei.value)

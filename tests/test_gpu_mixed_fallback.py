"""Mixed precision with its FP64 fallback: on a narrow window of the grid7 73^3
pencil (one of the serving stream's intervals) the poles lie so close to the
spectrum that the complex64 factors' refinement diverges; the query must notice
it at the first pole solve, run again with FP64 factors, say so in its stats,
and return the interval's eigenpairs to the usual bars (count = inertia count,
residual <= 1e-8, B-orthonormality <= 1e-10), the same eigenvalues as an FP64
query to 1e-10 relative.  Count and eigenvalues are the library's own at this
size (parity unpinned against the oracle; the FP64 path's parity is shown up to
64^3 elsewhere)."""
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


def test_mixed_falls_back_to_fp64(ctx):
    q = next(x for x in pencils.c4_stream(24, 0.5, seed=3, windows_per_pencil=3)
             if x["grid"] == 73 and x["window_id"] == 0)
    say(f"mixed query with FP64 fallback: grid7 73^3 interval ({q['a']:.9f}, {q['b']:.9f}), n_lambda {q['n_lambda']}")
    P = zolo.Pencil.from_grid(ctx, pencils.grid7(73), leaf_size=128)
    res = {}
    for prec in (zolo.ZOLO_PREC_MIXED, zolo.ZOLO_PREC_FP64):
        o = zolo.zolo_opts_default()
        o.r1, o.tol_gmres, o.max_subspace_iter, o.precision, o.tol_refine = 0, 1e-8, 4, prec, 1e-5
        eig, vec, st, rc = zolo.zolo_solve(ctx, P, q["a"], q["b"], q["n_lambda"], o)
        say(f"  precision {prec}: rc={rc} found {len(eig)} count {st['inertia_count']} resid {st['max_resid']:.2e} "
            f"fallback {st['precision_fallback']} b_orth {st['b_orth']:.1e}")
        assert rc == 0 and len(eig) == st["inertia_count"]
        assert st["max_resid"] <= 1e-8 and st["b_orth"] <= 1e-10
        res[prec] = (np.array(eig), st)
        del vec
    assert res[zolo.ZOLO_PREC_MIXED][1]["precision_fallback"] == 1
    assert res[zolo.ZOLO_PREC_FP64][1]["precision_fallback"] == 0
    e_m, e_d = res[zolo.ZOLO_PREC_MIXED][0], res[zolo.ZOLO_PREC_FP64][0]
    assert len(e_m) == len(e_d) and np.max(np.abs(e_m - e_d) / np.abs(e_d)) < 1e-10

"""Device Sylvester inertia (zolo_inertia) and eigengap estimation (zolo_solve
with NaN eigengaps and r1 = 0) against the oracle.

Inertia counts are integers and are compared exactly: against LAPACK's
eigenvalues on the dense 10^3 and 7x8x6 pencils, and against the oracle's
SuperLU symmetric-mode counts (oracle.sparse.inertia_neg) at 16^3 - 32^3.
Shifts are window ends (gap midpoints), so none lies near an eigenvalue.
"""
import json
import sys

import numpy as np
import pytest

import pencils
from oracle.dense import pencil_eigh_lapack
from oracle.sparse import inertia_neg
from oracle.subspace import b_orthonormality, inf_norm, rel_residuals

from .conftest import golden

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


def test_inertia_dense(ctx):
    for gen, shape in (("grid7", (10, 10, 10)), ("grid27p", (7, 8, 6))):
        say(f"inertia {gen} {shape} against LAPACK")
        gp = getattr(pencils, gen)(shape[0], ny=shape[1], nz=shape[2])
        A, B = gp.scipy()
        lam, _ = pencil_eigh_lapack(A.toarray(), B.toarray())
        idx = [3, 100, gp.n // 2, gp.n - 40]
        sig = np.array([0.5 * (lam[i] + lam[i + 1]) for i in idx] + [lam[0] - 1.0, lam[-1] + 1.0])
        P = zolo.Pencil.from_grid(ctx, gp, leaf_size=32)
        got = zolo.zolo_inertia(ctx, P, sig)
        ref = np.array([int(np.sum(lam < s)) for s in sig])
        say(f"  {got.tolist()} vs {ref.tolist()}")
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("gen,n", [("grid7", 16), ("grid7", 24), ("grid7", 32), ("grid27p", 24)])
def test_inertia_against_oracle(ctx, gen, n):
    w = json.load(open(golden(f"window_{gen}_{n}.json")))
    say(f"inertia {gen} {n}^3 against the oracle's SuperLU counts")
    gp = getattr(pencils, gen)(n)
    A, B = gp.scipy()
    ev = np.array(w["eigenvalues"])
    sig = np.array([w["a"], w["b"], 0.5 * (ev[10] + ev[11]), 0.5 * (ev[40] + ev[41])])
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=64)
    got = zolo.zolo_inertia(ctx, P, sig)
    ref = np.array([inertia_neg(A, B, float(s)) for s in sig])
    say(f"  {got.tolist()} vs {ref.tolist()}")
    assert np.array_equal(got, ref)
    assert got[1] - got[0] == len(ev)


@pytest.mark.parametrize("gen,n,nl", [("grid7", 10, 16), ("grid7", 24, 64), ("grid27p", 24, 64)])
def test_solve_estimated_gaps(ctx, gen, n, nl):
    """(a, b, n_lambda) only: eigengaps by inertia and r1 chosen by the library; the
    result must be the window the oracle stored (count, eigenvalues, residuals)."""
    w = json.load(open(golden(f"window_{gen}_{n}.json")))
    say(f"zolo_solve {gen} {n}^3 with estimated eigengaps and r1")
    gp = getattr(pencils, gen)(n)
    A, B = gp.scipy()
    P = zolo.Pencil.from_grid(ctx, gp, leaf_size=64)
    o = zolo.zolo_opts_default()
    o.r1 = 0
    o.max_subspace_iter = 6
    eig, vec, st, rc = zolo.zolo_solve(ctx, P, w["a"], w["b"], nl, o)
    say(f"  rc={rc} found={len(eig)} count={st['inertia_count']} r1={st['r1']} r2={st['r2']} l2={st['l2']:.3f} "
        f"gaps=({st['a_minus']:.6g}, {st['a_plus']:.6g}) ({st['b_minus']:.6g}, {st['b_plus']:.6g}) "
        f"t_gaps={st['t_gaps']:.3f}s iter={st['n_iter']} resid={st['max_resid']:.2e}")
    ref = np.array(w["eigenvalues"])
    assert rc == 0 and st["inertia_count"] == len(ref) == len(eig)
    assert st["a_minus"] < w["a"] < st["a_plus"] <= ref[0] and ref[-1] <= st["b_minus"] < w["b"] < st["b_plus"]
    eig = np.array(eig)
    assert np.max(np.abs(eig - ref) / np.abs(ref)) < 1e-10
    X = vec.cpu().numpy()
    assert np.max(rel_residuals(A, B, eig, X, inf_norm(A), inf_norm(B))) < 1e-8
    assert b_orthonormality(B, X) < 1e-10

"""GPU GenEO local eigenproblems and the GenEO two-level PCG (through the C ABI).

The GenEO eigenvalues are compared with the oracle's dense solve of the same
pencil (nu relative 1e-8); the PCG solution with the sparse direct fine solve
(energy-norm error <= 1e-6 at relative residual 1e-8).  Iteration counts are
reported, not compared: the condition bound of Sec. 3.2 has an unknown
constant (parity unpinned).
"""
import sys

import numpy as np
import pytest

from oracle import coarse, fem, geneo
from paper_2211_13893_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available(), "GPU tests need a GPU"
    return T


@pytest.mark.parametrize("case", ["beam", "cube"])
def test_geneo_eigs_and_pcg(torch, case):
    from paper_2211_13893_amd import msgfem
    if case == "beam":
        prob = synth.laminated_beam(n_ev=8)
    else:
        prob = synth.small_box(n=8, core=4, overlap=1, ovs=1, wrinkle=0.4, clamp=True, n_ev=8)
    say(f"[geneo] {case}: {prob.nsd} subdomains, n_ev 8")
    st = msgfem.LocalStage(prob, tol=1e-8, maxit=400, geneo=True)
    st.msgfem_assemble_local()
    out = st.msgfem_local_eigs()
    torch.cuda.synchronize()
    iters = out["iters"].cpu().numpy()
    say(f"  status {out['status'].cpu().numpy().tolist()} iterations {iters.tolist()} "
        f"max rho {[float(st.resid(out, b).max()) for b in range(len(st.batch))]}")
    assert int(out["status"].abs().sum()) == 0
    kec = fem.KeCache(prob)
    for b, j in enumerate(st.batch):
        lam_ref, *_ = geneo.geneo_local(prob, int(j), 8, kecache=kec)
        lam = st.eigvals(out, b).cpu().numpy()
        err = np.max(np.abs(1 / (lam + 1) - 1 / (lam_ref + 1)) * (lam_ref + 1))
        say(f"  sd {j}: GenEO nu rel err {err:.2e} ({iters[b]} LOBPCG iterations), lam {np.round(lam, 5).tolist()}")
        assert err <= 1e-8
    AH, bH = st.msgfem_coarse_assemble(out)
    res = st.msgfem_geneo_pcg(AH, rtol=1e-8, maxit=500)
    torch.cuda.synchronize()
    A = fem.assemble_global_sparse(prob)
    b = fem.traction_load(prob)
    uh = coarse.fine_solve(prob, A, b)
    e = coarse.energy_error(prob, A, uh, res["u"].cpu().numpy())
    say(f"  PCG: {res['iters']} iterations, relres {res['relres']:.2e}, energy error vs direct {e:.2e}")
    assert res["relres"] <= 1e-8
    assert int(res["status"].item()) == 0
    assert e <= 1e-6

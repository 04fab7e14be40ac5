"""GPU GenEO local eigenproblems and the GenEO two-level PCG (through the C ABI).

The GenEO eigenvalues are compared with the oracle's dense solve of the same
pencil (nu relative 1e-8); every GPU pair's residual is recomputed from the
oracle's matrices B = D A D and T = A + s B of the pencil (rho <= 1e-6 and
agreement with the library's rho), and the leading subspaces are held to the
Davis-Kahan bound formed from the same matrices; the PCG solution with the sparse direct fine solve
(energy-norm error <= 1e-6 at relative residual 1e-8).  Iteration counts are
reported, not compared: the condition bound of Sec. 3.2 has an unknown
constant (parity unpinned).
"""
import sys

import numpy as np
import pytest

from oracle import coarse, fem, geneo, gevp
from paper_2211_13893_amd import synth

import eigcheck

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
        lam_ref, phi_ref, gd, mu = geneo.geneo_local(prob, int(j), 12, kecache=kec)
        lam = st.eigvals(out, b).cpu().numpy()
        err = np.max(np.abs(1 / (lam + 1) - 1 / (lam_ref[:8] + 1)) * (lam_ref[:8] + 1))
        say(f"  sd {j}: GenEO nu rel err {err:.2e} ({iters[b]} LOBPCG iterations), lam {np.round(lam, 5).tolist()}")
        assert err <= 1e-8
        # the pencil's matrices on the non-Dirichlet DoFs of Omega_j
        elo, ehi = prob.omega_box(int(j))
        A = fem.assemble_box_dense(prob, elo, ehi, kec)
        keep = np.flatnonzero(prob.dirichlet[gd] == 0)
        Ak = A[np.ix_(keep, keep)]
        d = mu[keep]
        B = d[:, None] * Ak * d[None, :]
        T = Ak + 1.0 * B
        phi = st.eigvecs(out, b).cpu().numpy()
        X = phi[keep]
        nu = 1.0 / (lam + 1.0)
        r_or = np.array([gevp.nu_residual(B, T, float(nu[c]), X[:, c]) for c in range(8)])
        r_gpu = st.resid(out, b).cpu().numpy()
        say(f"    rho oracle max {r_or.max():.2e}, library max {r_gpu.max():.2e}")
        assert np.all(r_or <= 1e-6)
        assert np.all(np.abs(r_or - r_gpu) <= 1e-3 * np.maximum(r_or, r_gpu) + 1e-11)
        assert np.all(phi[np.flatnonzero(prob.dirichlet[gd] == 1)] == 0.0)
        nu_ref = 1.0 / (lam_ref + 1.0)
        gaps = (nu_ref[:8] - nu_ref[1:9]) / nu_ref[:8]
        for q in [c + 1 for c in range(8) if gaps[c] > 1e-3]:
            ang, bound = eigcheck.davis_kahan_mt(B, T, X[:, :q], phi_ref[keep][:, :q], float(nu_ref[q]))
            assert np.sin(ang) <= bound + 1e-10, (q, ang, bound)
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

"""Block-solve plan options against the oracle (through the C ABI).

Every combination of MSGFEM_OPT_SPLIT (one band, or nested dissection into
two chains and a separator Schur complement) and MSGFEM_OPT_SOLVE (vector
FMA; matrix cores with 8 or 16 columns per workgroup) must give the same
operators: on the beam's boxes, the interior solve A11^{-1} (op 2) and the
preconditioner (A + s D A D)^{-1} (op 3) against the oracle's dense solves
(rel 1e-9), and the local eigenpairs against the oracle's dense GEVP (nu rel
1e-8, oracle residual <= 1e-6).  The plan must report the layout it was asked
for (split boxes, solve family).  A tuned stage (the measured table's options
for its size class) is checked the same way.
"""
import sys

import numpy as np
import pytest

from oracle import fem, gevp
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


@pytest.fixture(scope="module")
def beam():
    prob = synth.laminated_beam()
    kec = fem.KeCache(prob)
    ops = {int(j): gevp.local_ops(prob, int(j), kec) for j in prob.batch}
    return prob, ops


COMBOS = [(0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3)]


def _family_expected(solve):
    return {1: 1, 2: 2, 3: 3}[solve]


@pytest.mark.parametrize("split,solve", COMBOS)
def test_apply_options(torch, beam, split, solve):
    from paper_2211_13893_amd import msgfem
    prob, dense = beam
    say(f"[options] beam apply, split {split}, solve {solve}")
    st = msgfem.LocalStage(prob, split=bool(split), solve=solve)
    fam = st.get_option(msgfem.INFO_SOLVE_FAMILY)
    nsplit = st.get_option(msgfem.INFO_SPLIT_BOXES)
    say(f"  families (A11 + 4 Ahat) {fam}, split boxes {nsplit}")
    assert fam % 4 == _family_expected(solve) and fam // 4 == _family_expected(solve)
    assert (nsplit > 0) == bool(split)
    st.msgfem_assemble_local()
    rng = np.random.default_rng(7)
    x = st.new_block()
    xs = []
    for b in range(len(st.batch)):
        xb = rng.standard_normal((st.boxes[b].n_dof, st.k))
        st.box_vector(x, b).copy_(torch.as_tensor(xb))
        xs.append(xb)
    y2 = st.msgfem_local_apply(2, x)
    y3 = st.msgfem_local_apply(3, x)
    torch.cuda.synchronize()
    for b, j in enumerate(st.batch):
        ops = dense[int(j)]
        cls, mu1 = ops.cls, ops.mu * (ops.cls == 1)
        keep = cls != 3
        A = ops.A
        i1 = np.flatnonzero(cls == 1)
        r2 = np.zeros_like(xs[b])
        r2[i1] = np.linalg.solve(A[np.ix_(i1, i1)], xs[b][i1])
        ia = np.flatnonzero(keep)
        Ah = A[np.ix_(ia, ia)] * (1.0 + np.outer(mu1[ia], mu1[ia]))
        r3 = np.zeros_like(xs[b])
        r3[ia] = np.linalg.solve(Ah, xs[b][ia])
        e2 = np.abs(st.box_vector(y2, b).cpu().numpy() - r2).max() / np.abs(r2).max()
        e3 = np.abs(st.box_vector(y3, b).cpu().numpy() - r3).max() / np.abs(r3).max()
        say(f"  box {b} (sd {j}): op 2 rel err {e2:.2e}, op 3 rel err {e3:.2e}")
        assert e2 <= 1e-9 and e3 <= 1e-9


def _eigs(torch, st, dense, n_ev):
    st.msgfem_assemble_local()
    out = st.msgfem_local_eigs()
    torch.cuda.synchronize()
    assert np.all(out["status"].cpu().numpy() == 0)
    for b, j in enumerate(st.batch):
        ops = dense[int(j)]
        ref = gevp.schur_gevp(ops, n_ev + 4)
        lam = st.eigvals(out, b).cpu().numpy()
        phi = st.eigvecs(out, b).cpu().numpy()
        err = np.max(np.abs(1.0 / (lam + 1.0) - ref.nu[:n_ev]) / ref.nu[:n_ev])
        r_or = eigcheck.oracle_rho(ref, ops.i2, lam, phi)
        say(f"  box {b} (sd {j}): nu rel err {err:.2e}, oracle rho {r_or.max():.2e}")
        assert err <= 1e-8 and r_or.max() <= 1e-6


@pytest.mark.parametrize("split,solve", [(0, 2), (1, 1), (1, 3)])
def test_eigs_options(torch, beam, split, solve):
    from paper_2211_13893_amd import msgfem
    prob, dense = beam
    say(f"[options] beam eigs, split {split}, solve {solve}")
    st = msgfem.LocalStage(prob, split=bool(split), solve=solve, tol=1e-9, maxit=400)
    _eigs(torch, st, dense, 10)


def test_eigs_tuned(torch, beam):
    from paper_2211_13893_amd import msgfem
    prob, dense = beam
    st = msgfem.LocalStage(prob, tuned=True, tol=1e-9, maxit=400)
    say(f"[options] beam eigs, tuned: class {st.size_class}, options {st.plan_options}")
    _eigs(torch, st, dense, 10)


def test_spmm_kernels_agree(torch):
    """MSGFEM_OPT_SPMM: the per-node kernel (1, and 0 on a batch of 16
    boxes) and the LDS-staged plane sweep (2) give the same stencil products
    (relative 1e-13: FP64 sums in another order); the plane sweep itself is
    checked against the oracle in test_gpu_local."""
    from paper_2211_13893_amd import msgfem
    say("[options] spmm kernels, 16 boxes of 9^3 nodes")
    prob = synth.uniform_batch(n_boxes=16, core=4, overlap=1, ovs=1, n_ev=4)
    st = msgfem.LocalStage(prob)
    assert st.get_option(msgfem.OPT_SPMM) == 0
    st.msgfem_assemble_local()
    x = st.new_block()
    x.normal_(generator=torch.Generator(device="cuda:0").manual_seed(4))
    out = {}
    for pref in (1, 2, 0):
        st.set_option(msgfem.OPT_SPMM, pref)
        out[pref] = [st.msgfem_local_apply(op, x).clone() for op in (0, 1)]
    torch.cuda.synchronize()
    for pref in (2, 0):
        for op in (0, 1):
            ref = out[1][op]
            e = float((out[pref][op] - ref).abs().max() / ref.abs().max())
            say(f"  spmm {pref} vs 1, op {op}: rel {e:.2e}")
            assert e <= 1e-13
    with pytest.raises(msgfem.MsgfemError):
        st.set_option(msgfem.OPT_SPMM, 3)


@pytest.mark.parametrize("name,split", [("beam", 1), ("beam", 0), ("uniform_16", 1)])
def test_chol_launches_agree(torch, name, split):
    """MSGFEM_OPT_CHOL: the tile Cholesky launched per step (1) and as one
    workgroup per matrix for all steps (2) run the same jobs with the same
    arithmetic, so the factors, and with them the interior solves (op 2:
    A11^{-1}, op 3: Ahat^{-1}) and the eigenpairs, are bitwise the same; the
    factor is checked against the oracle's solves in test_apply_options."""
    from paper_2211_13893_amd import msgfem
    prob = synth.laminated_beam() if name == "beam" else synth.uniform_batch(n_boxes=16)
    say(f"[options] Cholesky launches, {name}, split {split}")
    res = {}
    for pref in (msgfem.CHOL_STEPS, msgfem.CHOL_PER_MATRIX):
        st = msgfem.LocalStage(prob, chol=pref, split=bool(split))
        assert st.get_option(msgfem.OPT_CHOL) == pref
        st.msgfem_assemble_local()
        x = st.new_block()
        x.normal_(generator=torch.Generator(device="cuda:0").manual_seed(5))
        apply = [st.msgfem_local_apply(op, x).clone() for op in (2, 3)]
        out = st.msgfem_local_eigs()
        torch.cuda.synchronize()
        assert int(out["status"].abs().sum()) == 0
        res[pref] = (apply, out["evals"].clone(), out["iters"].clone())
        del st
    a, b = res[msgfem.CHOL_STEPS], res[msgfem.CHOL_PER_MATRIX]
    for op in (0, 1):
        assert torch.equal(a[0][op], b[0][op]), f"solve op {op + 2} differs"
    assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    st = msgfem.LocalStage(prob)
    assert st.get_option(msgfem.OPT_CHOL) == msgfem.CHOL_AUTO
    with pytest.raises(msgfem.MsgfemError):
        st.set_option(msgfem.OPT_CHOL, 3)

"""LOBPCG iterations replayed from HIP graphs against the eager loop (through the C ABI).

With MSGFEM_OPT_GRAPH = 1 the steady-state iterations of msgfem_local_eigs
are captured once per plan and buffer set and replayed; a box that converges
inside a replay is retired there, so every output (evals, evecs, resid,
iters, status) must equal the eager loop's bit for bit.  Checked on the beam
(one round), with n_ev 44 (a second, deflated round: six iterations per
replay), under precision 1, on a GenEO plan, for a masked subset solve, and
with maxit small enough that the last iterations and status bit 1 come from
the eager tail.  Each case alternates eager and graph calls on one plan
(three graph calls: the first captures, the later ones replay the cached
graph) and checks every graph call against the eager result.
"""
import sys

import numpy as np
import pytest

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


def _host(out):
    return {k: v.cpu().numpy().copy() for k, v in out.items()}


def _same(a, b):
    for key in ("evals", "evecs", "resid", "iters", "status"):
        x, y = a[key], b[key]
        if x.dtype == np.float64:
            x, y = x.view(np.int64), y.view(np.int64)
        if not np.array_equal(x, y):
            return key
    return None


def _run(st, mask=None):
    if mask is None:
        out = st.msgfem_local_eigs()
    else:
        # unselected boxes keep what the output holds: the same fill every call
        out = st.new_eig_output()
        for key in ("evals", "evecs", "resid"):
            out[key].fill_(-7.0)
        out["iters"].fill_(-7)
        out = st.msgfem_local_eigs_subset(mask, out)
    st.torch.cuda.synchronize()
    return _host(out)


def _compare(torch, st, mask=None):
    from paper_2211_13893_amd import msgfem
    st.msgfem_assemble_local()
    st.set_option(msgfem.OPT_GRAPH, 0)
    ref = _run(st, mask)
    assert st.get_option(msgfem.INFO_GRAPH_LAUNCHES) == 0
    x = st.new_block()
    x.normal_()
    for rep in range(3):
        st.set_option(msgfem.OPT_GRAPH, 1)
        got = _run(st, mask)
        launches = st.get_option(msgfem.INFO_GRAPH_LAUNCHES)
        its = st.get_option(msgfem.INFO_GRAPH_ITERS)
        cached = st.get_option(msgfem.INFO_GRAPHS_CACHED)
        say(f"  graph call {rep}: {launches} launches, {its} iterations, {cached} graphs cached, "
            f"iters {got['iters'].tolist()}, status {got['status'].tolist()}")
        bad = _same(ref, got)
        assert bad is None, f"graph call {rep}: {bad} differs from the eager loop"
        assert launches > 0 and cached >= 1
        # eager work on the same plan and buffers between the graph calls
        y = st.msgfem_local_apply(3, x)
        torch.cuda.synchronize()
        assert bool(torch.isfinite(y).all())
    st.set_option(msgfem.OPT_GRAPH, 0)
    assert st.get_option(msgfem.INFO_GRAPHS_CACHED) == 0
    again = _run(st, mask)
    assert _same(ref, again) is None
    return ref


def test_graph_beam(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] beam, n_ev 10, one round")
    st = msgfem.LocalStage(synth.laminated_beam(), tol=1e-9, maxit=400)
    ref = _compare(torch, st)
    assert np.all(ref["status"] == 0)


def test_graph_rounds(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] beam, n_ev 44: rounds of 24 and 20")
    st = msgfem.LocalStage(synth.laminated_beam(n_ev=44), tol=1e-6, maxit=400)
    ref = _compare(torch, st)
    assert np.all(ref["status"] == 0)


def test_graph_precision1_uniform(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] uniform batch, 4 boxes, precision 1")
    st = msgfem.LocalStage(synth.uniform_batch(n_boxes=4), tol=1e-6, maxit=200, precision=1)
    ref = _compare(torch, st)
    assert np.all(ref["status"] == 0)


def test_graph_geneo(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] beam, GenEO plan")
    st = msgfem.LocalStage(synth.laminated_beam(n_ev=8), tol=1e-8, maxit=400, geneo=True)
    ref = _compare(torch, st)
    assert np.all(ref["status"] == 0)


def test_graph_subset(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] beam, subset mask {1, 3}")
    st = msgfem.LocalStage(synth.laminated_beam(), tol=1e-9, maxit=400)
    _compare(torch, st, np.array([0, 1, 0, 1], np.int32))


def test_graph_maxit_tail(torch):
    from paper_2211_13893_amd import msgfem
    say("[graph] beam, maxit 9: replays for iterations 1-8, the last one eager")
    st = msgfem.LocalStage(synth.laminated_beam(), tol=1e-12, maxit=9)
    ref = _compare(torch, st)
    capped = (ref["status"] & 1) != 0
    assert capped.any() and np.all(ref["iters"][capped] == 9)

"""msgfem_local_apply_static (no work buffer, static scratch) against
msgfem_local_apply (caller work buffer) through the C ABI.

Both run the same kernels on the same inputs, so the outputs must agree bit
for bit, for every op, on two calls in a row with different plans, the
second plan smaller than the first (the static buffer keeps the first
call's contents, which the second call must not depend on).
"""
import ctypes
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


def _run(torch, st, seed):
    lib = st.lib
    x = st.new_block()
    x.normal_(generator=torch.Generator(device="cuda:0").manual_seed(seed))
    work = st._alloc_work()
    stream = torch.cuda.current_stream(st.device).cuda_stream
    for op in (0, 1, 2, 3):
        y_ref = torch.full_like(x, float("nan"))
        y_st = torch.full_like(x, float("nan"))
        rc = lib.msgfem_local_apply(st.plan, st.ops.data_ptr(), work.data_ptr(), op, st.k, x.data_ptr(),
                                    y_ref.data_ptr(), stream)
        assert rc == 0, lib.msgfem_plan_error(st.plan)
        rc = lib.msgfem_local_apply_static(st.plan, st.ops.data_ptr(), op, st.k, x.data_ptr(), y_st.data_ptr(),
                                           stream)
        assert rc == 0, lib.msgfem_plan_error(st.plan)
        torch.cuda.synchronize()
        assert torch.isfinite(y_ref).all()
        same = torch.equal(y_ref, y_st)
        say(f"  op {op}: {x.numel()} values, identical {same}")
        assert same


def test_static_apply_matches_work_buffer_apply(torch):
    from paper_2211_13893_amd import msgfem
    # first call: two uniform-batch boxes (10125 DoF each); second: the beam's
    # four smaller boxes
    say("[static apply] uniform batch, 2 boxes")
    big = msgfem.LocalStage(synth.uniform_batch(n_boxes=2))
    big.msgfem_assemble_local()
    _run(torch, big, 1)
    say("[static apply] beam, 4 boxes")
    small = msgfem.LocalStage(synth.laminated_beam())
    small.msgfem_assemble_local()
    assert small.sizes.n_dof < big.sizes.n_dof
    _run(torch, small, 2)

"""Plans driven from several host threads (through the C ABI).

The library keeps no per-call state outside a plan, and its one-time set-up
(the large-LDS kernel attributes) runs once whichever thread gets there
first.  Two plans on different batches, each on its own stream and its own
host thread, running assembly, factorisation and LOBPCG at the same time,
must give bit-identical eigenpairs, residuals and iteration counts to the
same plans run one after the other (every kernel sums in a fixed order), and
those eigenpairs must match the oracle's dense GEVP.
"""
import dataclasses
import sys
import threading

import numpy as np
import pytest

from oracle import fem, gevp
from paper_2211_13893_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_two_plans_two_threads():
    import torch
    from paper_2211_13893_amd import msgfem
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    prob = synth.laminated_beam()
    parts = [prob.batch[:2], prob.batch[2:]]
    probs = [dataclasses.replace(prob, batch=np.ascontiguousarray(b)) for b in parts]
    say("[threads] sequential reference, two plans of the beam's boxes")
    ref = []
    for p in probs:
        st = msgfem.LocalStage(p, tol=1e-6)
        st.msgfem_assemble_local()
        out = st.msgfem_local_eigs()
        torch.cuda.synchronize()
        ref.append({k: v.clone() for k, v in out.items() if torch.is_tensor(v)})
        del st
    stages = [msgfem.LocalStage(p, tol=1e-6) for p in probs]
    streams = [torch.cuda.Stream() for _ in stages]
    outs, errs = [None, None], []

    def work(i):
        try:
            with torch.cuda.stream(streams[i]):
                for _ in range(2):
                    stages[i].msgfem_assemble_local()
                    outs[i] = stages[i].msgfem_local_eigs()
                streams[i].synchronize()
        except Exception as e:   # reported by the main thread
            errs.append(repr(e))

    say("[threads] two plans, two streams, two host threads")
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=300)
    assert not any(t.is_alive() for t in th), "a thread did not finish"
    assert not errs, errs
    torch.cuda.synchronize()
    for i in range(2):
        for key in ("evals", "evecs", "resid", "iters", "status"):
            assert torch.equal(outs[i][key], ref[i][key]), (i, key)
        assert int(outs[i]["status"].abs().sum()) == 0
    kec = fem.KeCache(prob)
    for i, (st, p) in enumerate(zip(stages, probs)):
        for b, j in enumerate(st.batch):
            r = gevp.schur_gevp(gevp.local_ops(prob, int(j), kec), int(p.n_ev[j]))
            nu = 1.0 / (st.eigvals(outs[i], b).cpu().numpy() + 1.0)
            assert np.max(np.abs(nu - r.nu) / r.nu) <= 1e-8, (i, int(j))
    say("[threads] ok")

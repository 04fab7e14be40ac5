"""Adaptive local spaces by the eigenvalue threshold t (Sec. 1, Sec. 5).

The local space of subdomain j keeps the eigenpairs with lambda < 1/t, so the
number m_j is known only once an eigenvalue at or above 1/t has been computed.
Every subdomain starts with n_ev0 pairs; the boxes where all computed pairs
pass (status bit 16 of msgfem_select_modes) are solved again with twice as
many, up to n_ev_max (at most 48; the library computes more than 32 pairs
in deflated rounds), until an eigenvalue crosses 1/t or the cap is reached.
The final eigen output, in the layout of a plan with each box's last n_ev, is
merged from those solves by msgfem_merge_eigs and selected with t.  This
module only orchestrates: every array operation is a library call.
"""
from __future__ import annotations

import dataclasses
from typing import List

import numpy as np

from . import msgfem

# the library's cap on eigenpairs per box (beyond 32 they come in deflated rounds)
MAX_NEV = 48


@dataclasses.dataclass
class AdaptiveResult:
    stage: msgfem.LocalStage      # plan over the whole batch with the final n_ev per box
    eig: dict                     # its eigen output, merged from the solves
    selected: dict                # the same with the columns past m_j zeroed
    m: np.ndarray                 # m_j per batch box
    n_ev: np.ndarray              # eigenpairs computed per batch box
    capped: np.ndarray            # boxes where every computed pair passed at n_ev_max
    rounds: List[List[int]]       # subdomains solved in each round


def adaptive_local_spaces(problem, t: float, n_ev0: int = 8, n_ev_max: int = 48, **stage_kw) -> AdaptiveResult:
    if not t > 0:
        raise ValueError("threshold t must be positive")
    if not 1 <= n_ev0 <= n_ev_max <= MAX_NEV:
        raise ValueError(f"need 1 <= n_ev0 <= n_ev_max <= {MAX_NEV}")
    batch = [int(j) for j in problem.batch]
    nev = {j: n_ev0 for j in batch}
    solves, rounds = [], []
    todo = list(batch)
    while todo:
        st = msgfem.LocalStage(problem, batch=todo, n_ev=[nev[j] for j in todo], **stage_kw)
        st.msgfem_assemble_local()
        out = st.msgfem_local_eigs()
        _, sel = st.msgfem_select_modes(out, t)
        flags = sel["status"].cpu().numpy()
        if np.any(flags & 0b1101):
            raise msgfem.MsgfemError(f"local eigensolve failed, status {flags.tolist()}")
        again = [j for j, f in zip(todo, flags) if (f & 16) and nev[j] < n_ev_max]
        # boxes whose n_ev is final after this round
        keep = [b for b, j in enumerate(todo) if j not in again]
        solves.append((st, out, keep))
        rounds.append(list(todo))
        for j in again:
            nev[j] = min(2 * nev[j], n_ev_max)
        todo = again
    if len(solves) == 1:
        final, eig = solves[0][0], solves[0][1]
    else:
        final = msgfem.LocalStage(problem, batch=batch, n_ev=[nev[j] for j in batch], **stage_kw)
        final.msgfem_assemble_local()
        eig = final.new_eig_output()
        for st, out, keep in solves:
            eig = final.msgfem_merge_eigs(eig, st, out, boxes=keep)
    final.status.zero_()
    m, sel = final.msgfem_select_modes(eig, t)
    capped = (sel["status"].cpu().numpy() & 16) != 0
    return AdaptiveResult(final, eig, sel, m.cpu().numpy(), np.array([nev[j] for j in batch]), capped, rounds)

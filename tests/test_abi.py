"""The C ABI (include/msgfem.h) on the host: symbols, plan geometry, argument errors.

No GPU is needed: plan creation and the size/geometry queries are host-side.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import decomp
from paper_2211_13893_amd import msgfem, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(msgfem.LIB_PATH):
        pytest.skip("libmsgfem.so not built")
    return msgfem.load()


def test_library_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "msgfem.h")).read()
    names = sorted(set(re.findall(r"\b(msgfem_[a-z_]+)\s*\(", hdr)))
    assert "msgfem_local_eigs" in names and "msgfem_assemble_local" in names
    for n in names:
        assert hasattr(lib, n), n
    # the binding declares exactly the header's functions
    assert set(msgfem.SIGNATURES) == set(names)


def test_binding_option_codes_match_header():
    """Every plan option and counter code of the binding is the header's
    value, and the header has no option or counter the binding lacks."""
    hdr = open(os.path.join(ROOT, "include", "msgfem.h")).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define MSGFEM_((?:OPT|INFO)_[A-Z0-9_]+) (\d+)", hdr)}
    assert "OPT_CHOL" in codes and "INFO_MAX_BT_AHAT" in codes
    ours = {n: getattr(msgfem, n) for n in dir(msgfem) if re.fullmatch(r"(OPT|INFO)_[A-Z0-9_]+", n)}
    assert ours == codes


def _plan(prob, batch=None, n_ev=None, **kw):
    lib = _lib()
    mesh = msgfem.msgfem_mesh(prob.nx, prob.ny, prob.nz, prob.materials.shape[0], 1, 1, 1, 1)
    cores = np.ascontiguousarray(prob.cores, np.int32)
    ovs = np.ascontiguousarray(prob.ovs, np.int32)
    dec = msgfem.msgfem_decomp(prob.nsd, cores.ctypes.data, prob.overlap, ovs.ctypes.data)
    batch = np.asarray(prob.batch if batch is None else batch, np.int32)
    nev = np.asarray([prob.n_ev[j] for j in batch] if n_ev is None else n_ev, np.int32)
    opts = msgfem.msgfem_eig_opts(1.0, 1e-6, 100, kw.get("block", 0), kw.get("precision", 0), 0, 1)
    plan = ctypes.c_void_p()
    rc = lib.msgfem_plan_create(ctypes.byref(plan), 0, ctypes.byref(mesh), ctypes.byref(dec),
                                batch.ctypes.data, nev.ctypes.data, int(batch.size), ctypes.byref(opts))
    return lib, plan, rc, batch


def test_plan_geometry_matches_oracle_classes():
    for prob in (synth.laminated_beam(), synth.uniform_batch(n_boxes=3),
                 synth.small_box(n=8, core=2, overlap=1, ovs=1, clamp=True)):
        lib, plan, rc, batch = _plan(prob)
        assert rc == 0, lib.msgfem_plan_error(plan)
        s = msgfem.msgfem_sizes()
        assert lib.msgfem_plan_sizes(plan, ctypes.byref(s)) == 0
        assert s.n_box == batch.size
        tot = 0
        for b, j in enumerate(batch):
            bi = msgfem.msgfem_box_info()
            assert lib.msgfem_plan_box(plan, b, ctypes.byref(bi)) == 0
            cls = decomp.dof_classes(prob, int(j))
            elo, ehi = prob.omega_star_box(int(j))
            assert (bi.mx, bi.my, bi.mz) == tuple(int(ehi[d] - elo[d]) + 1 for d in range(3))
            assert bi.n_dof == cls.size
            # host count of interior-face DoFs = B2 plus Dirichlet DoFs lying on interior faces
            assert bi.n2 >= int((cls == 2).sum())
            assert bi.n2 + bi.n1 == cls.size
            tot += cls.size
        assert s.n_dof == tot
        assert s.block % 8 == 0 and s.block >= max(prob.n_ev[j] for j in batch)
        lib.msgfem_plan_destroy(plan)


def test_plan_rejects_bad_arguments():
    prob = synth.small_box(n=4, core=2, overlap=1, ovs=1)
    lib, plan, rc, _ = _plan(prob, batch=[0])
    # a 4^3 mesh covered by one oversampled box: no interior boundary, B2 empty
    assert rc == msgfem.MSGFEM_EARG
    assert b"B2 empty" in lib.msgfem_plan_error(plan)
    lib.msgfem_plan_destroy(plan)
    prob = synth.laminated_beam()
    lib, plan, rc, _ = _plan(prob, batch=[7], n_ev=[10])
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)
    lib, plan, rc, _ = _plan(prob, n_ev=[49, 10, 10, 10])
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)
    # more than 32 pairs: deflated rounds with block 32 (another block is refused)
    lib, plan, rc, _ = _plan(prob, n_ev=[40, 10, 10, 10])
    assert rc == 0
    s = msgfem.msgfem_sizes()
    assert lib.msgfem_plan_sizes(plan, ctypes.byref(s)) == 0 and s.block == 32
    lib.msgfem_plan_destroy(plan)
    lib, plan, rc, _ = _plan(prob, n_ev=[40, 10, 10, 10], block=24)
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)
    lib, plan, rc, _ = _plan(prob, precision=5)
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)
    # an empty batch and an odd block width are refused
    lib, plan, rc, _ = _plan(prob, batch=[], n_ev=[])
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)
    lib, plan, rc, _ = _plan(prob, block=13)
    assert rc == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)


def test_merge_eigs_rejects_mismatched_plans():
    """Host checks of msgfem_merge_eigs (no device work is reached): a source
    subdomain missing from the destination batch, another n_ev, another box."""
    prob = synth.laminated_beam()
    one = ctypes.c_void_p(256)
    ptrs = [one] * 8

    def merge(dst, src):
        return dst[0].msgfem_merge_eigs(dst[1], src[1], None, 0, *ptrs, None)

    full = _plan(prob)
    assert full[2] == 0
    part = _plan(prob, batch=[0, 2])
    sub = _plan(prob, batch=[1])
    sub_nev = _plan(prob, batch=[1], n_ev=[12])
    other = _plan(synth.laminated_beam(overlap=1), batch=[1])
    for p in (part, sub, sub_nev, other):
        assert p[2] == 0
    assert merge(part, sub) == msgfem.MSGFEM_EARG
    assert b"not in this plan's batch" in full[0].msgfem_plan_error(part[1])
    assert merge(full, sub_nev) == msgfem.MSGFEM_EARG
    assert merge(full, other) == msgfem.MSGFEM_EARG
    assert b"another box or n_ev" in full[0].msgfem_plan_error(full[1])
    assert merge(full, (None, None)) == msgfem.MSGFEM_EARG
    bad = (ctypes.c_int32 * 1)(5)
    assert full[0].msgfem_merge_eigs(full[1], sub[1], bad, 1, *ptrs, None) == msgfem.MSGFEM_EARG
    assert b"outside the source batch" in full[0].msgfem_plan_error(full[1])
    for p in (full, part, sub, sub_nev, other):
        p[0].msgfem_plan_destroy(p[1])


def test_subset_and_adaptive_reject_bad_arguments():
    """Host checks with no device work: msgfem_local_eigs_subset needs a mask;
    the adaptive driver needs t > 0 and 1 <= n_ev0 <= n_ev_max <= 32."""
    from paper_2211_13893_amd import adaptive
    prob = synth.laminated_beam()
    lib, plan, rc, _ = _plan(prob)
    assert rc == 0
    one = ctypes.c_void_p(256)
    assert lib.msgfem_local_eigs_subset(plan, one, one, None, None, one, one, one, one, one, None) \
        == msgfem.MSGFEM_EARG
    assert b"null mask" in lib.msgfem_plan_error(plan)
    lib.msgfem_plan_destroy(plan)
    for t, n0, nmax in ((0.0, 8, 32), (-1.0, 8, 32), (0.1, 0, 32), (0.1, 16, 8), (0.1, 8, 49)):
        with pytest.raises(ValueError):
            adaptive.adaptive_local_spaces(prob, t, n_ev0=n0, n_ev_max=nmax)


def test_static_apply_rejects_plans_beyond_its_scratch():
    # host-side check before any device work: the 64-box uniform batch needs far
    # more than the static buffer; a small plan fits
    lib = _lib()
    assert lib.msgfem_static_scratch_max() == 16 << 20
    prob = synth.uniform_batch(n_boxes=64)
    lib, plan, rc, _ = _plan(prob)
    assert rc == 0
    x = ctypes.c_void_p(1)
    y = ctypes.c_void_p(2)
    for op in (0, 3):
        r = lib.msgfem_local_apply_static(plan, ctypes.c_void_p(3), op, 32, x, y, None)
        assert r == msgfem.MSGFEM_ESIZE
        assert b"static buffer" in lib.msgfem_plan_error(plan)
    assert lib.msgfem_local_apply_static(plan, ctypes.c_void_p(3), 7, 32, x, y, None) == msgfem.MSGFEM_EARG
    lib.msgfem_plan_destroy(plan)

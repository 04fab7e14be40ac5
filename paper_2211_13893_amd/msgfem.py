"""Python binding of libmsgfem (the HIP library declared in include/msgfem.h).

Argument marshalling only: every computation runs in the library's HIP
kernels.  PyTorch provides device memory (the caller-owned buffers of the ABI)
and the stream.  Loading fails loudly when the library has not been built
(``python -m paper_2211_13893_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmsgfem.so")

MSGFEM_OK, MSGFEM_EARG, MSGFEM_EHIP, MSGFEM_ESIZE = 0, -1, -2, -3
OP_A, OP_DAD, OP_A11_SOLVE, OP_AHAT_SOLVE = 0, 1, 2, 3
STATUS_NOT_CONVERGED, STATUS_BAD_PIVOT, STATUS_NONFINITE = 1, 4, 8


class msgfem_mesh(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_mat", ctypes.c_int32), ("node_xyz", ctypes.c_void_p),
                ("elem_mat", ctypes.c_void_p), ("materials", ctypes.c_void_p),
                ("dirichlet", ctypes.c_void_p)]


class msgfem_decomp(ctypes.Structure):
    _fields_ = [("nsd", ctypes.c_int32), ("cores", ctypes.c_void_p),
                ("overlap", ctypes.c_int32), ("ovs", ctypes.c_void_p)]


class msgfem_eig_opts(ctypes.Structure):
    _fields_ = [("shift", ctypes.c_double), ("tol", ctypes.c_double), ("maxit", ctypes.c_int32),
                ("block", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("geneo", ctypes.c_int32), ("seed", ctypes.c_uint64)]


class msgfem_sizes(ctypes.Structure):
    _fields_ = [("ops_bytes", ctypes.c_int64), ("work_bytes", ctypes.c_int64),
                ("n_eval", ctypes.c_int64), ("n_evec", ctypes.c_int64), ("n_dof", ctypes.c_int64),
                ("block", ctypes.c_int32), ("n_box", ctypes.c_int32)]


class msgfem_box_info(ctypes.Structure):
    _fields_ = [("sd", ctypes.c_int32), ("mx", ctypes.c_int32), ("my", ctypes.c_int32),
                ("mz", ctypes.c_int32), ("g0", ctypes.c_int32 * 3), ("n_nodes", ctypes.c_int32),
                ("n_dof", ctypes.c_int32), ("n_ev", ctypes.c_int32), ("n1", ctypes.c_int32),
                ("n2", ctypes.c_int32), ("n3", ctypes.c_int32),
                ("stencil_off", ctypes.c_int64), ("cls_off", ctypes.c_int64),
                ("mu_off", ctypes.c_int64), ("vec_off", ctypes.c_int64),
                ("evec_off", ctypes.c_int64), ("eval_off", ctypes.c_int64)]


class msgfem_load(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("face", ctypes.c_void_p), ("g", ctypes.c_void_p)]


class msgfem_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


# plan option keys (msgfem.h)
OPT_GRAPH = 1
OPT_SPLIT = 2
OPT_SOLVE = 3
OPT_SPMM = 4
SPMM_AUTO, SPMM_NODES, SPMM_PLANES = 0, 1, 2   # values of OPT_SPMM
OPT_CHOL = 5
CHOL_AUTO, CHOL_STEPS, CHOL_PER_MATRIX = 0, 1, 2   # values of OPT_CHOL
INFO_GRAPH_LAUNCHES = 100
INFO_GRAPH_ITERS = 101
INFO_GRAPHS_CACHED = 102
INFO_SPLIT_BOXES = 103
INFO_SOLVE_FAMILY = 104
INFO_MAX_BT_A11 = 105
INFO_MAX_BT_AHAT = 106

_P = ctypes.c_void_p
SIGNATURES = {
    "msgfem_plan_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int,
                                          ctypes.POINTER(msgfem_mesh), ctypes.POINTER(msgfem_decomp),
                                          _P, _P, ctypes.c_int32, ctypes.POINTER(msgfem_eig_opts)]),
    "msgfem_plan_destroy": (None, [_P]),
    "msgfem_plan_error": (ctypes.c_char_p, [_P]),
    "msgfem_plan_sizes": (ctypes.c_int, [_P, ctypes.POINTER(msgfem_sizes)]),
    "msgfem_plan_box": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(msgfem_box_info)]),
    "msgfem_assemble_local": (ctypes.c_int, [_P, _P, _P, _P]),
    "msgfem_local_eigs": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "msgfem_local_eigs_subset": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "msgfem_local_apply": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "msgfem_local_apply_static": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P]),
    "msgfem_static_scratch_max": (ctypes.c_int64, []),
    "msgfem_select_modes": (ctypes.c_int, [_P, _P, _P, ctypes.c_double, _P, _P, _P, _P, _P]),
    "msgfem_error_norms": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, _P, _P]),
    "msgfem_box_digest": (ctypes.c_int, [_P, _P, _P, _P]),
    "msgfem_merge_eigs": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "msgfem_coarse_sizes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "msgfem_coarse_assemble": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(msgfem_load), _P, _P, _P, _P,
                                              _P, _P]),
    "msgfem_coarse_solve": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "msgfem_pcg_sizes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "msgfem_geneo_pcg": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.POINTER(msgfem_load), ctypes.c_double,
                                        ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_double), _P, _P]),
    "msgfem_coarse_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(msgfem_mesh),
                                            ctypes.POINTER(msgfem_decomp), _P, ctypes.c_int32]),
    "msgfem_coarse_destroy": (None, [_P]),
    "msgfem_coarse_error": (ctypes.c_char_p, [_P]),
    "msgfem_coarse_store_sizes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                                 ctypes.POINTER(ctypes.c_int32)]),
    "msgfem_coarse_box": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "msgfem_coarse_add": (ctypes.c_int, [_P, _P, _P, _P, ctypes.POINTER(msgfem_load), _P, _P, _P]),
    "msgfem_coarse_galerkin": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "msgfem_coarse_solve_store": (ctypes.c_int, [_P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "msgfem_coarse_pcg_sizes": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "msgfem_coarse_pcg": (ctypes.c_int, [_P, _P, _P, ctypes.POINTER(msgfem_load), ctypes.c_double, ctypes.c_int32,
                                         _P, _P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                                         _P, _P]),
    "msgfem_coarse_energy": (ctypes.c_int, [_P, _P, _P, _P, _P, _P]),
    "msgfem_plan_set_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int64]),
    "msgfem_plan_get_option": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "msgfem_profile": (ctypes.c_int, [_P, ctypes.c_int32]),
    "msgfem_profile_stats": (ctypes.c_int, [_P, ctypes.POINTER(msgfem_kernel_stat), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
    "msgfem_warm_features": (ctypes.c_int, [_P, _P, _P, _P]),
    "msgfem_warm_basis": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, _P, _P]),
    "msgfem_warm_labels": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          _P, _P]),
    "msgfem_warm_start": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_uint64, _P, _P]),
    "msgfem_cnn_sizes": (ctypes.c_int, [ctypes.c_int32] * 5 + [ctypes.POINTER(ctypes.c_int64)] * 2),
    "msgfem_cnn_forward": (ctypes.c_int, [_P] + [ctypes.c_int32] * 6 + [_P, _P, _P, _P]),
    "msgfem_cnn_backward": (ctypes.c_int, [_P] + [ctypes.c_int32] * 6 + [_P, _P, _P, _P]),
    "msgfem_cnn_loss": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                       _P, _P, _P]),
    "msgfem_cnn_adam": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, _P]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libmsgfem.so and declare its C signatures (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2211_13893_amd.build`")
    # torch first: the library must bind to the HIP runtime torch loads (a
    # second runtime loaded on the library's own dependency finds no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MsgfemError(RuntimeError):
    pass


def _check(rc: int, plan=None, what: str = ""):
    if rc != MSGFEM_OK:
        msg = ""
        if plan:
            m = load().msgfem_plan_error(plan)
            msg = m.decode() if m else ""
        raise MsgfemError(f"{what} failed with code {rc}: {msg}")


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else 0


def _stream_handle(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class LocalStage:
    """One plan of the local spectral stage: a mesh, its decomposition and a batch.

    ``problem`` is a :class:`paper_2211_13893_amd.synth.Problem`.  Device
    copies of the mesh arrays are kept for the plan's lifetime.
    """

    def __init__(self, problem, batch: Optional[Sequence[int]] = None,
                 n_ev: Optional[Sequence[int]] = None, device: str = "cuda:0", shift: float = 1.0,
                 tol: float = 1e-6, maxit: int = 200, block: int = 0, seed: int = 1234,
                 geneo: bool = False, precision: int = 0, graph: Optional[bool] = None,
                 split: Optional[bool] = None, solve: Optional[int] = None, tuned: bool = False,
                 spmm: Optional[int] = None, chol: Optional[int] = None):
        import torch
        self.torch = torch
        lib = load()
        self.lib = lib
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise MsgfemError("LocalStage needs a GPU device")
        dev = self.device
        p = problem
        self.problem = p
        self.batch = np.asarray(p.batch if batch is None else batch, dtype=np.int32)
        nev = np.asarray([int(p.n_ev[j]) for j in self.batch] if n_ev is None else n_ev, dtype=np.int32)
        self.n_ev = nev
        self._xyz = torch.as_tensor(np.ascontiguousarray(p.xyz, dtype=np.float64), device=dev)
        self._emat = torch.as_tensor(np.ascontiguousarray(p.elem_mat, dtype=np.int32), device=dev)
        self._mats = torch.as_tensor(np.ascontiguousarray(p.materials, dtype=np.float64), device=dev)
        self._dir = torch.as_tensor(np.ascontiguousarray(p.dirichlet, dtype=np.uint8), device=dev)
        self.mesh = msgfem_mesh(p.nx, p.ny, p.nz, p.materials.shape[0], _ptr(self._xyz),
                                _ptr(self._emat), _ptr(self._mats), _ptr(self._dir))
        self._cores = np.ascontiguousarray(p.cores, dtype=np.int32)
        self._ovs = np.ascontiguousarray(p.ovs, dtype=np.int32)
        dec = msgfem_decomp(p.nsd, self._cores.ctypes.data, p.overlap, self._ovs.ctypes.data)
        opts = msgfem_eig_opts(shift, tol, maxit, block, precision, 1 if geneo else 0, seed)
        self.precision = precision
        self.geneo = geneo
        self.shift = shift
        plan = _P()
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        rc = lib.msgfem_plan_create(ctypes.byref(plan), idx, ctypes.byref(self.mesh),
                                    ctypes.byref(dec), self.batch.ctypes.data, nev.ctypes.data,
                                    int(self.batch.size), ctypes.byref(opts))
        self.plan = plan
        _check(rc, plan, "msgfem_plan_create")
        # plan options: the measured table for the plan's size class (tuned),
        # then explicit arguments; the factor layout (split, solve family) is
        # fixed before the sizes are read and buffers allocated
        opts_set = {}
        if tuned:
            from . import tuning
            s0 = msgfem_sizes()
            _check(lib.msgfem_plan_sizes(plan, ctypes.byref(s0)), plan, "msgfem_plan_sizes")
            bt = ctypes.c_int64()
            _check(lib.msgfem_plan_get_option(plan, INFO_MAX_BT_AHAT, ctypes.byref(bt)), plan, "msgfem_plan_get_option")
            self.size_class = tuning.size_class(int(bt.value), int(s0.n_box), int(s0.block))
            table = tuning.options_for(self.size_class) or {}
            if geneo:
                # a GenEO coarse store fixes the interior band layout (default split and family)
                table = {key: v for key, v in table.items() if key == "graph"}
            opts_set.update(table)
        for key, val in (("split", split), ("solve", solve), ("graph", graph), ("spmm", spmm), ("chol", chol)):
            if val is not None:
                opts_set[key] = int(val)
        self.plan_options = dict(opts_set)
        for key, code in (("split", OPT_SPLIT), ("solve", OPT_SOLVE), ("graph", OPT_GRAPH), ("spmm", OPT_SPMM),
                          ("chol", OPT_CHOL)):
            if key in opts_set:
                _check(lib.msgfem_plan_set_option(plan, code, int(opts_set[key])), plan, "msgfem_plan_set_option")
        s = msgfem_sizes()
        _check(lib.msgfem_plan_sizes(plan, ctypes.byref(s)), plan, "msgfem_plan_sizes")
        self.sizes = s
        self.k = s.block
        self.boxes = []
        for b in range(self.batch.size):
            bi = msgfem_box_info()
            _check(lib.msgfem_plan_box(plan, b, ctypes.byref(bi)), plan, "msgfem_plan_box")
            self.boxes.append(bi)
        self.ops = None
        self.work = None

    def load_mesh(self, problem):
        """Copy the mesh arrays (node coordinates, element materials, material
        table, Dirichlet flags) of `problem` into this stage's device arrays,
        which the plan reads at every msgfem_assemble_local.  The problem must
        have this plan's geometry: mesh size, material count, decomposition and
        batch (only the values change, e.g. another wrinkle or layup), so the
        plan, its ops and work buffers are reused as they are."""
        torch = self.torch
        p, q = problem, self.problem
        same = ((p.nx, p.ny, p.nz, p.materials.shape[0], p.overlap) == (q.nx, q.ny, q.nz, q.materials.shape[0],
                                                                      q.overlap)
                and np.array_equal(p.cores, q.cores) and np.array_equal(p.ovs, q.ovs)
                and np.array_equal(np.asarray(p.batch), np.asarray(q.batch))
                and np.array_equal(np.asarray(p.n_ev), np.asarray(q.n_ev)))
        if not same:
            raise MsgfemError("load_mesh needs a problem with this plan's mesh size, materials count, "
                              "decomposition and batch")
        for dst, src, dt in ((self._xyz, p.xyz, np.float64), (self._emat, p.elem_mat, np.int32),
                             (self._mats, p.materials, np.float64), (self._dir, p.dirichlet, np.uint8)):
            a = torch.as_tensor(np.ascontiguousarray(src, dtype=dt))
            if a.numel() != dst.numel():
                raise MsgfemError("load_mesh: array sizes differ")
            dst.copy_(a.view(dst.shape))
        self.problem = p

    def set_option(self, key: int, value: int):
        """msgfem_plan_set_option"""
        _check(self.lib.msgfem_plan_set_option(self.plan, int(key), int(value)), self.plan, "msgfem_plan_set_option")

    def get_option(self, key: int) -> int:
        """msgfem_plan_get_option"""
        v = ctypes.c_int64()
        _check(self.lib.msgfem_plan_get_option(self.plan, int(key), ctypes.byref(v)), self.plan,
               "msgfem_plan_get_option")
        return int(v.value)

    def __del__(self):
        try:
            if getattr(self, "plan", None):
                self.lib.msgfem_plan_destroy(self.plan)
                self.plan = None
        except Exception:
            pass

    # -- buffers -------------------------------------------------------
    def _alloc_ops(self):
        if self.ops is None:
            self.ops = self.torch.empty(self.sizes.ops_bytes, dtype=self.torch.uint8, device=self.device)
        return self.ops

    def _alloc_work(self):
        if self.work is None:
            self.work = self.torch.empty(self.sizes.work_bytes, dtype=self.torch.uint8, device=self.device)
        return self.work

    # -- ABI calls -----------------------------------------------------
    def msgfem_assemble_local(self, status=None):
        torch = self.torch
        ops = self._alloc_ops()
        if status is None:
            status = torch.zeros(len(self.batch), dtype=torch.int32, device=self.device)
        rc = self.lib.msgfem_assemble_local(self.plan, _ptr(ops), _ptr(status),
                                            _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_assemble_local")
        self.status = status
        return status

    def msgfem_local_eigs(self, x0=None, out=None):
        torch = self.torch
        if self.ops is None:
            raise MsgfemError("assemble first")
        work = self._alloc_work()
        s = self.sizes
        nb = len(self.batch)
        if out is None:
            out = dict(evals=torch.empty(s.n_eval, dtype=torch.float64, device=self.device),
                       evecs=torch.empty(s.n_evec, dtype=torch.float64, device=self.device),
                       resid=torch.empty(s.n_eval, dtype=torch.float64, device=self.device),
                       iters=torch.empty(nb, dtype=torch.int32, device=self.device))
        rc = self.lib.msgfem_local_eigs(self.plan, _ptr(self.ops), _ptr(work), _ptr(x0),
                                        _ptr(out["evals"]), _ptr(out["evecs"]), _ptr(out["resid"]),
                                        _ptr(out["iters"]), _ptr(self.status),
                                        _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_local_eigs")
        out["status"] = self.status
        return out

    def _check_eig_output(self, out, what: str):
        """An eigen output in this stage's layout: float64 evals/evecs/resid and int32
        iters, contiguous, on this stage's device, of this plan's lengths (the
        kernels write through these pointers, so a stored output of another plan
        must not reach them)."""
        torch = self.torch
        s = self.sizes
        want = {"evals": (torch.float64, s.n_eval), "evecs": (torch.float64, s.n_evec),
                "resid": (torch.float64, s.n_eval), "iters": (torch.int32, s.n_box)}
        for key, (dt, n) in want.items():
            t = out.get(key) if isinstance(out, dict) else None
            if t is None:
                raise MsgfemError(f"{what}: output '{key}' missing")
            on_dev = t.device.type == "cuda" and (self.device.index is None or t.device.index == self.device.index)
            if t.dtype != dt or not t.is_contiguous() or not on_dev or t.numel() != n:
                raise MsgfemError(f"{what}: '{key}' must be a contiguous {dt} tensor of {n} elements on "
                                  f"{self.device} (got {t.dtype}, {t.numel()} elements on {t.device})")

    def msgfem_local_eigs_subset(self, mask, out, x0=None):
        """Solves only the boxes with mask[b] != 0, writing their slots of the
        eigen output `out` (this stage's layout) in place; the other boxes keep
        what `out` holds (msgfem_local_eigs_subset)."""
        torch = self.torch
        if self.ops is None:
            raise MsgfemError("assemble first")
        if hasattr(mask, "cpu"):          # a torch tensor, e.g. digests compared on the device
            mask = mask.cpu().numpy()
        m = np.ascontiguousarray(mask, dtype=np.int32)
        if m.shape != (len(self.batch),):
            raise MsgfemError(f"mask needs one entry per batch box ({len(self.batch)})")
        self._check_eig_output(out, "msgfem_local_eigs_subset")
        md = torch.tensor(m, dtype=torch.int32, device=self.device)
        work = self._alloc_work()
        rc = self.lib.msgfem_local_eigs_subset(self.plan, _ptr(self.ops), _ptr(work), _ptr(x0), _ptr(md),
                                               _ptr(out["evals"]), _ptr(out["evecs"]), _ptr(out["resid"]),
                                               _ptr(out["iters"]), _ptr(self.status),
                                               _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_local_eigs_subset")
        out["status"] = self.status
        return out

    def msgfem_local_apply(self, op: int, x, k: Optional[int] = None):
        torch = self.torch
        k = self.k if k is None else k
        y = torch.zeros_like(x)
        work = self._alloc_work()
        rc = self.lib.msgfem_local_apply(self.plan, _ptr(self.ops), _ptr(work), op, k, _ptr(x), _ptr(y),
                                         _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_local_apply")
        return y

    def msgfem_local_apply_static(self, op: int, x, y=None, k: Optional[int] = None):
        """msgfem_local_apply with the library's static scratch (no work buffer)."""
        torch = self.torch
        k = self.k if k is None else k
        y = torch.zeros_like(x) if y is None else y
        rc = self.lib.msgfem_local_apply_static(self.plan, _ptr(self.ops), op, k, _ptr(x), _ptr(y),
                                                _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_local_apply_static")
        return y

    def msgfem_coarse_sizes(self):
        nb = ctypes.c_int64()
        nh = ctypes.c_int32()
        _check(self.lib.msgfem_coarse_sizes(self.plan, ctypes.byref(nb), ctypes.byref(nh)), self.plan,
               "msgfem_coarse_sizes")
        return nb.value, nh.value

    def msgfem_select_modes(self, eig_out, t: float):
        """Adaptive local spaces (msgfem_select_modes): per box the eigenpairs
        with lambda < 1/t.  Returns (m, a copy of eig_out whose eigenvectors
        have the other columns zeroed, ready for msgfem_coarse_assemble)."""
        torch = self.torch
        nb = len(self.batch)
        m = torch.empty(nb, dtype=torch.int32, device=self.device)
        sel = dict(eig_out)
        sel["evecs"] = torch.empty_like(eig_out["evecs"])
        rc = self.lib.msgfem_select_modes(self.plan, _ptr(self.ops), _ptr(eig_out["evals"]), float(t),
                                          _ptr(eig_out["evecs"]), _ptr(sel["evecs"]), _ptr(m),
                                          _ptr(self.status), _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_select_modes")
        sel["status"] = self.status
        return m, sel

    def msgfem_error_norms(self, u_ref, u):
        """Error metrics of Sec. 5.3 (msgfem_error_norms): a device double[6] with
        the four integrals and e_d, e_eps."""
        torch = self.torch
        for name, x in (("u_ref", u_ref), ("u", u)):
            on_dev = x.device.type == "cuda" and (self.device.index is None or x.device.index == self.device.index)
            if x.dtype != torch.float64 or not x.is_contiguous() or not on_dev:
                raise MsgfemError(f"{name} must be a contiguous float64 tensor on {self.device}")
        if u_ref.numel() != u.numel():
            raise MsgfemError("u_ref and u differ in length")
        out = torch.empty(6, dtype=torch.float64, device=self.device)
        rc = self.lib.msgfem_error_norms(self.plan, _ptr(u_ref), _ptr(u), int(u.numel()), _ptr(out),
                                         _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_error_norms")
        return out

    def msgfem_box_digest(self):
        """Per-box 64-bit digests of the assembled local eigenproblems
        (msgfem_box_digest), as a device int64 tensor (same bits as uint64)."""
        torch = self.torch
        if self.ops is None:
            raise MsgfemError("assemble first")
        d = torch.empty(len(self.batch), dtype=torch.int64, device=self.device)
        rc = self.lib.msgfem_box_digest(self.plan, _ptr(self.ops), _ptr(d), _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_box_digest")
        return d

    def new_eig_output(self):
        """A zeroed eigen output in this stage's msgfem_local_eigs layout."""
        torch = self.torch
        s = self.sizes
        return dict(evals=torch.zeros(s.n_eval, dtype=torch.float64, device=self.device),
                    evecs=torch.zeros(s.n_evec, dtype=torch.float64, device=self.device),
                    resid=torch.zeros(s.n_eval, dtype=torch.float64, device=self.device),
                    iters=torch.zeros(s.n_box, dtype=torch.int32, device=self.device),
                    status=self.status)

    def msgfem_merge_eigs(self, stored, src_stage, src_out, boxes=None):
        """Returns a copy of `stored` (an eigen output of this stage's layout) with
        the boxes of `src_stage` (all, or the batch positions `boxes`) replaced by
        `src_out` (msgfem_merge_eigs)."""
        torch = self.torch
        self._check_eig_output(stored, "msgfem_merge_eigs (stored)")
        src_stage._check_eig_output(src_out, "msgfem_merge_eigs (source)")
        out = {k: (v if k == "status" else v.clone()) for k, v in stored.items()}
        sel = None if boxes is None else np.ascontiguousarray(boxes, dtype=np.int32)
        rc = self.lib.msgfem_merge_eigs(self.plan, src_stage.plan, None if sel is None else sel.ctypes.data,
                                        0 if sel is None else int(sel.size),
                                        _ptr(src_out["evals"]), _ptr(src_out["evecs"]),
                                        _ptr(src_out["resid"]), _ptr(src_out["iters"]), _ptr(out["evals"]),
                                        _ptr(out["evecs"]), _ptr(out["resid"]), _ptr(out["iters"]),
                                        _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_merge_eigs")
        return out

    def msgfem_coarse_assemble(self, eig_out):
        torch = self.torch
        nbytes, nh = self.msgfem_coarse_sizes()
        if getattr(self, "coarse", None) is None or self.coarse.numel() < nbytes:
            self.coarse = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        ld = self._load()
        AH = torch.empty((nh, nh), dtype=torch.float64, device=self.device)
        bH = torch.empty(nh, dtype=torch.float64, device=self.device)
        rc = self.lib.msgfem_coarse_assemble(self.plan, _ptr(self.ops), _ptr(self._alloc_work()),
                                             ctypes.byref(ld), _ptr(eig_out["evecs"]), _ptr(self.coarse),
                                             _ptr(AH), _ptr(bH), _ptr(self.status),
                                             _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_coarse_assemble")
        return AH, bH

    def msgfem_coarse_solve(self, AH, bH):
        torch = self.torch
        nh = AH.shape[0]
        c = torch.empty(nh, dtype=torch.float64, device=self.device)
        ng = self.problem.n_dofs
        uG = torch.empty(ng, dtype=torch.float64, device=self.device)
        up = torch.empty(ng, dtype=torch.float64, device=self.device)
        st = torch.zeros(1, dtype=torch.int32, device=self.device)
        rc = self.lib.msgfem_coarse_solve(self.plan, _ptr(self.ops), _ptr(self._alloc_work()),
                                          _ptr(self.coarse), _ptr(AH), _ptr(bH), _ptr(c), _ptr(uG), _ptr(up),
                                          _ptr(st), _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_coarse_solve")
        return dict(c=c, uG=uG, up=up, status=st)

    def _load(self):
        faces = {"x-": 0, "x+": 1, "y-": 2, "y+": 3, "z-": 4, "z+": 5}
        tr = self.problem.tractions
        self._face = np.asarray([faces[f] for f, _ in tr], dtype=np.int32)
        self._g = np.ascontiguousarray(np.asarray([g for _, g in tr], dtype=np.float64).reshape(-1, 3))
        return msgfem_load(len(tr), self._face.ctypes.data if len(tr) else 0,
                           self._g.ctypes.data if len(tr) else 0)

    def msgfem_geneo_pcg(self, AH, rtol: float = 1e-8, maxit: int = 1000, u0=None):
        torch = self.torch
        nbytes = ctypes.c_int64()
        _check(self.lib.msgfem_pcg_sizes(self.plan, ctypes.byref(nbytes)), self.plan, "msgfem_pcg_sizes")
        if getattr(self, "pcg_ws", None) is None or self.pcg_ws.numel() < nbytes.value:
            self.pcg_ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        u = torch.zeros(self.problem.n_dofs, dtype=torch.float64, device=self.device) if u0 is None else u0.clone()
        it = ctypes.c_int32()
        rel = ctypes.c_double()
        st = torch.zeros(1, dtype=torch.int32, device=self.device)
        ld = self._load()
        rc = self.lib.msgfem_geneo_pcg(self.plan, _ptr(self.ops), _ptr(self._alloc_work()), _ptr(self.coarse),
                                       _ptr(AH), ctypes.byref(ld), rtol, maxit, _ptr(self.pcg_ws), _ptr(u),
                                       ctypes.byref(it), ctypes.byref(rel), _ptr(st),
                                       _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_geneo_pcg")
        return dict(u=u, iters=it.value, relres=rel.value, status=st)

    def msgfem_profile(self, enable: bool):
        _check(self.lib.msgfem_profile(self.plan, 1 if enable else 0), self.plan, "msgfem_profile")

    def msgfem_profile_stats(self):
        n = ctypes.c_int32()
        arr = (msgfem_kernel_stat * 16)()
        _check(self.lib.msgfem_profile_stats(self.plan, arr, 16, ctypes.byref(n)), self.plan,
               "msgfem_profile_stats")
        return {arr[i].name.decode(): dict(launches=arr[i].launches, ms=arr[i].ms,
                                           bytes=arr[i].bytes, flops=arr[i].flops)
                for i in range(min(n.value, 16))}

    # -- learned warm start ---------------------------------------------
    def msgfem_warm_features(self):
        """Network input [n_box, 6, ez, ey, ex] (float32) of every box."""
        torch = self.torch
        bi = self.boxes[0]
        feat = torch.empty((len(self.batch), 6, bi.mz - 1, bi.my - 1, bi.mx - 1), dtype=torch.float32,
                           device=self.device)
        rc = self.lib.msgfem_warm_features(self.plan, _ptr(self.ops), _ptr(feat),
                                           _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_warm_features")
        return feat

    def msgfem_warm_basis(self, eig_out, ng: int):
        """Basis G [n_dof, ng] (float64) from box 0's eigenvectors."""
        torch = self.torch
        G = torch.empty((self.boxes[0].n_dof, ng), dtype=torch.float64, device=self.device)
        rc = self.lib.msgfem_warm_basis(self.plan, _ptr(self.ops), _ptr(eig_out["evecs"]), ng, _ptr(G),
                                        _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_warm_basis")
        return G

    def msgfem_warm_labels(self, eig_out, G, ne: int):
        """Label projectors [n_box, ng, ng] (float32)."""
        torch = self.torch
        ng = G.shape[1]
        P = torch.empty((len(self.batch), ng, ng), dtype=torch.float32, device=self.device)
        rc = self.lib.msgfem_warm_labels(self.plan, _ptr(self.ops), _ptr(eig_out["evecs"]), _ptr(G.contiguous()),
                                         G.shape[0], ng, ne, _ptr(P), _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_warm_labels")
        return P

    def msgfem_warm_start(self, coef, G, ne: int, seed: int = 0):
        """Start block (flat [sum n_dof * k], float64) for msgfem_local_eigs."""
        torch = self.torch
        x0 = self.new_block()
        rc = self.lib.msgfem_warm_start(self.plan, _ptr(self.ops), _ptr(coef.contiguous()), _ptr(G.contiguous()),
                                        G.shape[0], G.shape[1], ne, seed, _ptr(x0),
                                        _stream_handle(torch, self.device))
        _check(rc, self.plan, "msgfem_warm_start")
        return x0

    # -- views ---------------------------------------------------------
    def stencil(self, b: int):
        bi = self.boxes[b]
        n = bi.n_nodes * 243 * 8
        return self.ops[bi.stencil_off:bi.stencil_off + n].view(self.torch.float64).view(243, bi.n_nodes)

    def classes(self, b: int):
        bi = self.boxes[b]
        return self.ops[bi.cls_off:bi.cls_off + bi.n_dof]

    def mu(self, b: int):
        bi = self.boxes[b]
        return self.ops[bi.mu_off:bi.mu_off + 8 * bi.n_dof].view(self.torch.float64)

    def box_vector(self, vec, b: int, k: Optional[int] = None):
        """View of box b inside a block vector [sum n_dof][k] (flat)."""
        k = self.k if k is None else k
        bi = self.boxes[b]
        return vec[bi.vec_off:bi.vec_off + bi.n_dof * k].view(bi.n_dof, k)

    def new_block(self, k: Optional[int] = None):
        k = self.k if k is None else k
        return self.torch.zeros(self.sizes.n_dof * k, dtype=self.torch.float64, device=self.device)

    def eigvals(self, out, b: int):
        bi = self.boxes[b]
        return out["evals"][bi.eval_off:bi.eval_off + bi.n_ev]

    def eigvecs(self, out, b: int):
        bi = self.boxes[b]
        return out["evecs"][bi.evec_off:bi.evec_off + bi.n_dof * bi.n_ev].view(bi.n_dof, bi.n_ev)

    def resid(self, out, b: int):
        bi = self.boxes[b]
        return out["resid"][bi.eval_off:bi.eval_off + bi.n_ev]


class CoarseStore:
    """The coarse problem of one decomposition gathered across plans
    (msgfem_coarse_*): ``add`` every plan's eigen output, then ``galerkin``,
    ``solve`` (MS-GFEM) or, for a GenEO store, ``pcg`` and ``energy``.

    Keeps device copies of the mesh arrays and the store buffer."""

    def __init__(self, problem, geneo: bool = False, n_ev: Optional[Sequence[int]] = None, device: str = "cuda:0"):
        import torch
        self.torch = torch
        lib = load()
        self.lib = lib
        self.device = torch.device(device)
        p = problem
        self.problem = p
        self.geneo = geneo
        dev = self.device
        self._xyz = torch.as_tensor(np.ascontiguousarray(p.xyz, dtype=np.float64), device=dev)
        self._emat = torch.as_tensor(np.ascontiguousarray(p.elem_mat, dtype=np.int32), device=dev)
        self._mats = torch.as_tensor(np.ascontiguousarray(p.materials, dtype=np.float64), device=dev)
        self._dir = torch.as_tensor(np.ascontiguousarray(p.dirichlet, dtype=np.uint8), device=dev)
        self.mesh = msgfem_mesh(p.nx, p.ny, p.nz, p.materials.shape[0], _ptr(self._xyz), _ptr(self._emat),
                                _ptr(self._mats), _ptr(self._dir))
        self._cores = np.ascontiguousarray(p.cores, dtype=np.int32)
        self._ovs = np.ascontiguousarray(p.ovs, dtype=np.int32)
        dec = msgfem_decomp(p.nsd, self._cores.ctypes.data, p.overlap, self._ovs.ctypes.data)
        self.n_ev = np.ascontiguousarray(p.n_ev if n_ev is None else n_ev, dtype=np.int32)
        h = _P()
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        rc = lib.msgfem_coarse_create(ctypes.byref(h), idx, ctypes.byref(self.mesh), ctypes.byref(dec),
                                      self.n_ev.ctypes.data, 1 if geneo else 0)
        self.h = h
        self._check(rc, "msgfem_coarse_create")
        nb, nh, kc = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(lib.msgfem_coarse_store_sizes(h, ctypes.byref(nb), ctypes.byref(nh), ctypes.byref(kc)),
                    "msgfem_coarse_store_sizes")
        self.store_bytes, self.NH, self.kc = nb.value, nh.value, kc.value
        self.store = torch.empty(self.store_bytes, dtype=torch.uint8, device=dev)
        self.pcg_ws = None

    def _check(self, rc, what):
        if rc != MSGFEM_OK:
            m = self.lib.msgfem_coarse_error(self.h) if getattr(self, "h", None) else b""
            raise MsgfemError(f"{what} failed with code {rc}: {m.decode() if m else ''}")

    def __del__(self):
        try:
            if getattr(self, "h", None):
                self.lib.msgfem_coarse_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def _stream(self):
        return _stream_handle(self.torch, self.device)

    def add(self, stage: "LocalStage", eig_out):
        ld = stage._load()
        rc = self.lib.msgfem_coarse_add(self.h, stage.plan, _ptr(stage.ops), _ptr(stage._alloc_work()), ctypes.byref(ld),
                                        _ptr(eig_out["evecs"]), _ptr(self.store), self._stream())
        self._check(rc, "msgfem_coarse_add")

    def galerkin(self):
        torch = self.torch
        AH = torch.empty((self.NH, self.NH), dtype=torch.float64, device=self.device)
        bH = torch.empty(self.NH, dtype=torch.float64, device=self.device)
        self._check(self.lib.msgfem_coarse_galerkin(self.h, _ptr(self.store), _ptr(AH), _ptr(bH), self._stream()),
                    "msgfem_coarse_galerkin")
        return AH, bH

    def solve(self, AH, bH):
        torch = self.torch
        n = self.problem.n_dofs
        c = torch.empty(self.NH, dtype=torch.float64, device=self.device)
        uG = torch.empty(n, dtype=torch.float64, device=self.device)
        up = torch.empty(n, dtype=torch.float64, device=self.device)
        st = torch.zeros(1, dtype=torch.int32, device=self.device)
        rc = self.lib.msgfem_coarse_solve_store(self.h, _ptr(self.store), _ptr(AH), _ptr(bH), _ptr(c), _ptr(uG),
                                                _ptr(up), _ptr(st), self._stream())
        self._check(rc, "msgfem_coarse_solve_store")
        return dict(c=c, uG=uG, up=up, status=st)

    def _load(self):
        faces = {"x-": 0, "x+": 1, "y-": 2, "y+": 3, "z-": 4, "z+": 5}
        tr = self.problem.tractions
        self._face = np.asarray([faces[f] for f, _ in tr], dtype=np.int32)
        self._g = np.ascontiguousarray(np.asarray([g for _, g in tr], dtype=np.float64).reshape(-1, 3))
        return msgfem_load(len(tr), self._face.ctypes.data if len(tr) else 0, self._g.ctypes.data if len(tr) else 0)

    def pcg(self, A0, rtol: float = 1e-8, maxit: int = 1000, u0=None):
        torch = self.torch
        nb = ctypes.c_int64()
        self._check(self.lib.msgfem_coarse_pcg_sizes(self.h, ctypes.byref(nb)), "msgfem_coarse_pcg_sizes")
        if self.pcg_ws is None or self.pcg_ws.numel() < nb.value:
            self.pcg_ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        u = torch.zeros(self.problem.n_dofs, dtype=torch.float64, device=self.device) if u0 is None else u0.clone()
        it, rel = ctypes.c_int32(), ctypes.c_double()
        st = torch.zeros(1, dtype=torch.int32, device=self.device)
        ld = self._load()
        rc = self.lib.msgfem_coarse_pcg(self.h, _ptr(self.store), _ptr(A0), ctypes.byref(ld), rtol, maxit,
                                        _ptr(self.pcg_ws), _ptr(u), ctypes.byref(it), ctypes.byref(rel), _ptr(st),
                                        self._stream())
        self._check(rc, "msgfem_coarse_pcg")
        return dict(u=u, iters=it.value, relres=rel.value, status=st)

    def energy(self, u_ref, u):
        """[(u_ref-u)^T A (u_ref-u), u_ref^T A u_ref] (device float64[2]) after ``pcg``."""
        torch = self.torch
        if self.pcg_ws is None:
            raise MsgfemError("energy needs the workspace of a completed pcg")
        out = torch.empty(2, dtype=torch.float64, device=self.device)
        self._check(self.lib.msgfem_coarse_energy(self.h, _ptr(self.pcg_ws), _ptr(u_ref), _ptr(u), _ptr(out),
                                                  self._stream()), "msgfem_coarse_energy")
        return out

    def box(self, sd: int):
        off, n, row = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        self._check(self.lib.msgfem_coarse_box(self.h, sd, ctypes.byref(off), ctypes.byref(n), ctypes.byref(row)),
                    "msgfem_coarse_box")
        return off.value, n.value, row.value


# -- the warm-start network (plan-independent) ---------------------------------
def msgfem_cnn_sizes(cin: int, width: int, n_out: int, d: int, batch: int):
    """(n_params, work_bytes) of the network for this batch size."""
    n = ctypes.c_int64()
    w = ctypes.c_int64()
    _check(load().msgfem_cnn_sizes(cin, width, n_out, d, batch, ctypes.byref(n), ctypes.byref(w)), None,
           "msgfem_cnn_sizes")
    return n.value, w.value


def _dev_stream(t):
    import torch
    return _stream_handle(torch, t.device)


def msgfem_cnn_forward(params, cin: int, width: int, n_out: int, x, bf16: bool, work):
    """Network output [batch, n_out] (float32) for x [batch, cin, d, d, d]."""
    import torch
    b, d = x.shape[0], x.shape[2]
    out = torch.empty((b, n_out), dtype=torch.float32, device=x.device)
    rc = load().msgfem_cnn_forward(_ptr(params), cin, width, n_out, d, b, 1 if bf16 else 0,
                                   _ptr(x.contiguous()), _ptr(out), _ptr(work), _dev_stream(x))
    _check(rc, None, "msgfem_cnn_forward")
    return out


def msgfem_cnn_backward(params, cin: int, width: int, n_out: int, d: int, gout, bf16: bool, work):
    """Parameter gradient (float32, n_params) of sum(gout * out)."""
    import torch
    grads = torch.empty_like(params)
    rc = load().msgfem_cnn_backward(_ptr(params), cin, width, n_out, d, gout.shape[0], 1 if bf16 else 0,
                                    _ptr(gout.contiguous()), _ptr(grads), _ptr(work), _dev_stream(gout))
    _check(rc, None, "msgfem_cnn_backward")
    return grads


def msgfem_cnn_loss(out, labels, ng: int, ne: int, gscale: float = 1.0):
    """(loss per sample [batch], gscale * its gradient [batch, ng*ne])."""
    import torch
    b = out.shape[0]
    loss = torch.empty(b, dtype=torch.float32, device=out.device)
    gout = torch.empty_like(out)
    rc = load().msgfem_cnn_loss(_ptr(out.contiguous()), _ptr(labels.contiguous()), ng, ne, b, gscale,
                                _ptr(loss), _ptr(gout), _dev_stream(out))
    _check(rc, None, "msgfem_cnn_loss")
    return loss, gout


def msgfem_cnn_adam(params, grads, m, v, step: int, lr: float):
    """One Adam step, in place on params, m and v."""
    rc = load().msgfem_cnn_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(), step, lr,
                                _dev_stream(params))
    _check(rc, None, "msgfem_cnn_adam")

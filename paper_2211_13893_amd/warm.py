"""Learned warm start of the local eigensolver (an addition to the method).

The paper solves every local GEVP (Sec. 3.3, matrix form Sec. 4.3) from
scratch.  Here a small 3D CNN, run by the library's own kernels, predicts the
low eigenspace of an oversampled box from its element field, and the
prediction seeds the LOBPCG block:

* basis: G = the ng lowest A-harmonic eigenvectors of a homogeneous
  isotropic reference box with the same node grid, orthonormal on B2
  (``msgfem_warm_basis``);
* labels: the projector P_b onto G^T X_b for the box's first ne
  eigenvectors X_b (``msgfem_warm_labels``), computed by the FP64 path;
* network: coefficients C_b (ng x ne) = CNN(features_b), trained with the
  rotation-invariant loss |C C^T - P|_F^2 (``msgfem_cnn_*``);
* start: X0 = G C on B2 plus Gaussian guard columns (``msgfem_warm_start``),
  with a Gaussian column wherever a prediction is zero or not finite.

Everything here is orchestration: every array operation runs in libmsgfem.
"""
from __future__ import annotations

from typing import Optional

import numpy as np

from . import msgfem, synth

CIN = 6          # feature channels (msgfem_warm_features)


def init_params(cin: int, width: int, n_out: int, seed: int) -> np.ndarray:
    """Flat float32 parameter vector in the library's layout: He-normal
    convolution weights, zero biases, a 1/sqrt(width)-scaled affine map."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([17, seed])))
    parts = []
    c = cin
    for _ in range(4):
        parts.append(rng.standard_normal(width * c * 27) * np.sqrt(2.0 / (27 * c)))
        parts.append(np.zeros(width))
        c = width
    parts.append(rng.standard_normal(n_out * width) * np.sqrt(1.0 / width))
    parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def reference_basis(ng: int = 32, device: str = "cuda:0", core: int = 8, overlap: int = 1, ovs: int = 2):
    """G [n_dof, ng] (float64, device) from a homogeneous isotropic box of the
    warm-start grid, without a wrinkle."""
    p = synth.warm_start_batch(n_boxes=1, homogeneous=True, wrinkle_max=0.0, core=core, overlap=overlap,
                               ovs=ovs, n_ev=ng)
    st = msgfem.LocalStage(p, device=device)
    st.msgfem_assemble_local()
    out = st.msgfem_local_eigs()
    G = st.msgfem_warm_basis(out, ng)
    return G, st, out


class WarmStartNet:
    """The network's parameters and Adam state on the device."""

    def __init__(self, ng: int = 32, ne: int = 16, width: int = 32, d: int = 14, bf16: bool = True,
                 seed: int = 0, device: str = "cuda:0"):
        import torch
        self.torch = torch
        self.ng, self.ne, self.width, self.d, self.bf16 = ng, ne, width, d, bf16
        self.n_out = ng * ne
        self.device = torch.device(device)
        p = init_params(CIN, width, self.n_out, seed)
        n_params, _ = msgfem.msgfem_cnn_sizes(CIN, width, self.n_out, d, 1)
        assert p.size == n_params
        self.params = torch.as_tensor(p, device=self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step = 0
        self._work = None
        self._work_batch = 0

    def _work_for(self, batch: int):
        if self._work is None or self._work_batch < batch:
            _, wb = msgfem.msgfem_cnn_sizes(CIN, self.width, self.n_out, self.d, batch)
            self._work = self.torch.empty(wb, dtype=self.torch.uint8, device=self.device)
            self._work_batch = batch
        return self._work

    def forward(self, feat):
        return msgfem.msgfem_cnn_forward(self.params, CIN, self.width, self.n_out, feat, self.bf16,
                                         self._work_for(feat.shape[0]))

    def train_step(self, feat, labels, lr: float = 1e-3) -> float:
        """One Adam step on the mean loss of the batch; returns that mean."""
        work = self._work_for(feat.shape[0])
        out = msgfem.msgfem_cnn_forward(self.params, CIN, self.width, self.n_out, feat, self.bf16, work)
        loss, gout = msgfem.msgfem_cnn_loss(out, labels, self.ng, self.ne, 1.0 / feat.shape[0])
        grads = msgfem.msgfem_cnn_backward(self.params, CIN, self.width, self.n_out, self.d, gout, self.bf16,
                                           work)
        self.step += 1
        msgfem.msgfem_cnn_adam(self.params, grads, self.m, self.v, self.step, lr)
        return float(loss.cpu().numpy().astype(np.float64).mean())

    def start_block(self, stage, G, feat=None, seed: int = 0):
        """Warm start block of a LocalStage whose boxes have this grid."""
        if feat is None:
            feat = stage.msgfem_warm_features()
        coef = self.forward(feat)
        return stage.msgfem_warm_start(coef, G, self.ne, seed)


def training_set(seed: int, G, ne: int = 16, n_boxes: int = 64, device: str = "cuda:0",
                 stage_kw: Optional[dict] = None):
    """Features and labels of one seeded warm-start batch, the labels from the
    FP64 path; also the stage's random-start iteration counts."""
    p = synth.warm_start_batch(n_boxes=n_boxes, seed=seed)
    st = msgfem.LocalStage(p, device=device, **(stage_kw or {}))
    st.msgfem_assemble_local()
    out = st.msgfem_local_eigs()
    feat = st.msgfem_warm_features()
    P = st.msgfem_warm_labels(out, G, ne)
    return feat, P, out, st


def fit(G, seeds=range(4), steps: int = 300, lr: float = 2e-3, ne: int = 16, bf16: bool = True,
        net_seed: int = 1, device: str = "cuda:0", n_boxes: int = 64):
    """Train a network on the warm-start batches of `seeds` (labels from the
    FP64 path): `steps` Adam steps on one batch each, drawn in a seeded
    order, lr dropped 4x for the last 30%.  Returns (net, last losses)."""
    data = []
    for s in seeds:
        feat, P, _, st = training_set(int(s), G, ne=ne, n_boxes=n_boxes, device=device)
        data.append((feat, P))
        del st
    net = WarmStartNet(ng=G.shape[1], ne=ne, bf16=bf16, seed=net_seed, device=device)
    order = np.random.Generator(np.random.PCG64(np.random.SeedSequence([19, net_seed]))).integers(
        len(data), size=steps)
    losses = []
    for i, b in enumerate(order):
        losses.append(net.train_step(*data[int(b)], lr=lr if i < 0.7 * steps else lr / 4))
    return net, losses


def dataset(G, seeds, ne: int = 16, n_boxes: int = 256, device: str = "cuda:0", log=None):
    """Features and labels (FP64 path) of the warm-start batches of `seeds`,
    n_boxes boxes each.  The batches share their geometry, so one plan is
    reused and only the mesh arrays change between them (LocalStage.load_mesh)."""
    import torch
    feats, labels = [], []
    st = None
    for i, s in enumerate(seeds):
        if log and i % 8 == 0:
            log(f"  warm-start data: batch {i + 1}/{len(seeds)} (seed {s})")
        p = synth.warm_start_batch(n_boxes=n_boxes, seed=int(s))
        if st is None:
            st = msgfem.LocalStage(p, device=device, tuned=True)
        else:
            st.load_mesh(p)
        st.msgfem_assemble_local()
        out = st.msgfem_local_eigs()
        feats.append(st.msgfem_warm_features())
        labels.append(st.msgfem_warm_labels(out, G, ne))
        del out
    del st
    torch.cuda.empty_cache()
    return feats, labels


def fit_dataset(G, feats, labels, steps: int = 2000, lr: float = 2e-3, ne: int = 16, bf16: bool = True,
                net_seed: int = 1, minibatch: int = 64, device: str = "cuda:0", log=None):
    """Adam on minibatches of `minibatch` boxes drawn (seeded) from the whole
    data set; lr dropped 4x for the last 30%.  Returns (net, losses)."""
    net = WarmStartNet(ng=G.shape[1], ne=ne, bf16=bf16, seed=net_seed, device=device)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([23, net_seed])))
    losses = []
    for i in range(steps):
        j = int(rng.integers(len(feats)))
        nb = feats[j].shape[0]
        o = int(rng.integers(max(1, nb // minibatch))) * minibatch
        f, p = feats[j][o:o + minibatch], labels[j][o:o + minibatch]
        losses.append(net.train_step(f, p, lr=lr if i < 0.7 * steps else lr / 4))
        if log and (i + 1) % 250 == 0:
            log(f"  warm-start training: step {i + 1}/{steps}, loss {np.mean(losses[-50:]):.3f}")
    return net, losses


def evaluate(net, G, seeds, ne: int = 16, n_boxes: int = 256, device: str = "cuda:0", log=None):
    """On the held-out batches of `seeds`: LOBPCG iterations and seconds per
    batch from the random start and from the network's start (its features,
    inference and start block inside the timed region), and the largest
    relative difference of nu between the two.  Returns a dict of arrays."""
    import time
    import torch
    it_r, it_w, t_r, t_w, dnu, ok = [], [], [], [], [], True
    st = None
    for i, s in enumerate(seeds):
        if log:
            log(f"  warm-start held-out batch {i + 1}/{len(seeds)} (seed {s})")
        p = synth.warm_start_batch(n_boxes=n_boxes, seed=int(s))
        if st is None:
            st = msgfem.LocalStage(p, device=device, tuned=True)
            st.msgfem_assemble_local()
            st.msgfem_local_eigs()          # first calls: buffers allocated outside the timings
            net.start_block(st, G)
        else:
            st.load_mesh(p)
        st.msgfem_assemble_local()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out_r = st.msgfem_local_eigs()
        torch.cuda.synchronize()
        t_r.append(time.perf_counter() - t0)
        it_r.append(out_r["iters"].cpu().numpy())
        lam_r = out_r["evals"].cpu().numpy()
        ok &= bool(np.all(out_r["status"].cpu().numpy() == 0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out_w = st.msgfem_local_eigs(x0=net.start_block(st, G))
        torch.cuda.synchronize()
        t_w.append(time.perf_counter() - t0)
        it_w.append(out_w["iters"].cpu().numpy())
        lam_w = out_w["evals"].cpu().numpy()
        ok &= bool(np.all(out_w["status"].cpu().numpy() == 0))
        nu_r, nu_w = 1.0 / (lam_r + 1.0), 1.0 / (lam_w + 1.0)
        dnu.append(float(np.abs(nu_w - nu_r).max() / nu_r.max()))
        del out_r, out_w
    del st
    torch.cuda.empty_cache()
    return {"iters_random": np.concatenate(it_r), "iters_warm": np.concatenate(it_w),
            "seconds_random": np.array(t_r), "seconds_warm": np.array(t_w), "max_nu_rel_diff": max(dnu),
            "all_converged": ok}

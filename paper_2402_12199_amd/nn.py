"""Drivers of the network kernels: autograd wrapper, labelling with the bead
sum, normalisation constants and the training loop.

All arithmetic runs in the HIP kernels behind `abi`; this module only
allocates device buffers, slices batches and loops.
"""
from __future__ import annotations

import numpy as np
import torch

from . import abi


def make_norm(d_cut: float, e_shift: float = 0.0, e_scale: float = 1.0, d_gain: float = 2.3,
              q_gain: float = 2.0) -> np.ndarray:
    """16 normalisation numbers: in_shift[7], in_scale[7], out_shift, out_scale.

    The network sees (d_gain d / d_cut, q_gain q): with d uniform in direction
    and |d| <= d_cut, and q uniform on S^3 (components of standard deviation
    1/2), these gains give inputs of about unit spread.  It predicts
    (E - e_shift) / e_scale.
    """
    return np.concatenate([np.zeros(7), [d_gain / d_cut] * 3 + [q_gain] * 4, [e_shift, e_scale]]).astype(np.float32)


def make_norm_sym(d_cut: float, e_shift: float = 0.0, e_scale: float = 1.0, d_gain: float = 2.3) -> np.ndarray:
    """Normalisation of the symmetry-reduced cube-pair descriptor
    (p_x, p_y, p_z, w_y, w_z, cos 4 a3, sin 4 a3): the centre coordinates as
    in make_norm, w_y, w_z (|w_y|, |w_z| <= 0.82) and the unit circle of
    4 a3 at about unit spread."""
    shift = [0.0] * 7
    scale = [d_gain / d_cut] * 3 + [2.0, 2.0, 1.0, 1.0]
    return np.concatenate([shift, scale, [e_shift, e_scale]]).astype(np.float32)


def make_norm_features(s: np.ndarray, e_shift: float = 0.0, e_scale: float = 1.0) -> np.ndarray:
    """Normalisation of a reduced descriptor from its training values s
    (P, 7): each used input shifted by its mean and scaled to unit spread;
    inputs that are identically zero stay zero."""
    s = np.asarray(s, np.float64)
    mean, std = s.mean(0), s.std(0)
    used = std > 0
    shift = np.where(used, mean, 0.0)
    scale = np.where(used, 1.0 / np.where(used, std, 1.0), 0.0)
    return np.concatenate([shift, scale, [e_shift, e_scale]]).astype(np.float32)


def sym_descriptors(desc: torch.Tensor, chunk: int = 1 << 18, with_jac: bool = True, form: str = "cube"):
    """(sym (7, P), jac (49, P) or None) of pair descriptors desc (7, P) on
    the device (rb_cube_sym_descriptors, or rb_cyl_sym_descriptors for
    form="cyl"), in chunks when the Jacobian is dropped."""
    fn = {"cube": abi.rb_cube_sym_descriptors, "cyl": abi.rb_cyl_sym_descriptors}[form]
    P = desc.shape[1]
    sym = torch.empty((7, P), dtype=torch.float32, device=desc.device)
    if with_jac:
        jac = torch.empty((49, P), dtype=torch.float32, device=desc.device)
        fn(desc, sym, jac)
        return sym, jac
    for s0 in range(0, P, chunk):
        d = desc[:, s0:s0 + chunk].contiguous()
        m = d.shape[1]
        sy = torch.empty((7, m), dtype=torch.float32, device=desc.device)
        jc = torch.empty((49, m), dtype=torch.float32, device=desc.device)
        fn(d, sy, jc)
        sym[:, s0:s0 + m] = sy
    return sym, None


class NNPairEnergy(torch.autograd.Function):
    """E = g_NN(desc) with a hand-written input gradient.

    desc: (7, P) float32 CUDA tensor (structure of arrays).  Forward calls
    rb_nn_pair_eval; backward calls rb_nn_pair_grad with the incoming
    gradient as the reverse-pass seed.  The parameters are constants here
    (training uses rb_nn_train_step).
    """

    @staticmethod
    def forward(ctx, desc, params, norm, precision):
        desc = desc.contiguous()
        E = torch.empty(desc.shape[1], dtype=torch.float32, device=desc.device)
        abi.rb_nn_pair_eval(params, norm, precision, desc, E)
        ctx.save_for_backward(desc, params)
        ctx.norm = norm
        ctx.precision = precision
        return E

    @staticmethod
    def backward(ctx, gE):
        desc, params = ctx.saved_tensors
        g = torch.empty_like(desc)
        abi.rb_nn_pair_grad(params, ctx.norm, ctx.precision, desc, gE.contiguous().float(), None, g, None)
        return g, None, None, None


def nn_pair_energy(desc, params, norm, precision=abi.RB_PREC_BF16):
    return NNPairEnergy.apply(desc, params, norm, precision)


def label_pairs(ctx: abi.Ctx, desc: np.ndarray, type_i: int = 0, type_j: int = 0, chunk: int = 1 << 20,
                device="cuda") -> np.ndarray:
    """Bead-sum labels (P, 11) = E, F_j, tau_i, tau_j, r_min for desc (P, 7)."""
    P = len(desc)
    out = np.empty((P, 11), dtype=np.float32)
    for s in range(0, P, chunk):
        d = torch.tensor(np.ascontiguousarray(desc[s:s + chunk].T, dtype=np.float32), device=device)
        o = torch.empty((11, d.shape[1]), dtype=torch.float32, device=device)
        abi.rb_bead_pair_eval(ctx, d, type_i, type_j, o)
        out[s:s + chunk] = o.cpu().numpy().T
    return out


class Trainer:
    """Adam on the FP32 master parameters with the energy loss, on the GPU."""

    def __init__(self, params: np.ndarray, norm: np.ndarray, precision=abi.RB_PREC_BF16, batch=8192, lr=1e-3,
                 beta1=0.9, beta2=0.999, eps=1e-8, device="cuda", fm: dict | None = None):
        """fm: dict(lam_f, lam_t) adds force and torque matching
        (rb_nn_train_step_fm); the data then need (6, n) F_j, tau_j labels."""
        self.dev = torch.device(device)
        self.params = torch.tensor(np.asarray(params, np.float32), device=self.dev)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.norm = np.asarray(norm, np.float32)
        self.precision = precision
        self.batch = batch
        self.lr, self.beta1, self.beta2, self.eps = lr, beta1, beta2, eps
        self.t = 0
        self.fm = fm
        nws = abi.rb_nn_train_fm_workspace_bytes(batch) if fm else abi.rb_nn_train_workspace_bytes(batch)
        self.ws = torch.zeros(nws, dtype=torch.uint8, device=self.dev)
        self.loss = torch.zeros(2, dtype=torch.float32, device=self.dev)   # energy, matching

    def step(self, desc, labels, idx, grad_out=None, loss=None, ft=None):
        """One Adam step on the batch idx; the batch losses go to `loss` (a
        two-element device tensor, default self.loss: energy, matching)."""
        self.t += 1
        loss = self.loss if loss is None else loss
        if self.fm is None:
            abi.rb_nn_train_step(self.params, self.m, self.v, self.t, self.norm, self.precision, idx.numel(), desc,
                                 labels, idx, self.lr, self.beta1, self.beta2, self.eps, loss[:1], grad_out, self.ws)
        else:
            abi.rb_nn_train_step_fm(self.params, self.m, self.v, self.t, self.norm, self.precision, idx.numel(),
                                    desc, labels, ft, idx, self.fm["lam_f"], self.fm["lam_t"], self.lr, self.beta1,
                                    self.beta2, self.eps, loss, grad_out, self.ws)

    def epoch(self, desc, labels, g: np.random.Generator, ft=None):
        """One pass over the data in a random order; returns the mean energy
        loss (the mean matching loss is left in self.fm_loss).  Each step
        writes its losses into its own slots, so the loop launches nothing
        but the training step."""
        n = labels.numel()
        perm = torch.tensor(g.permutation(n).astype(np.int32), device=self.dev)
        nb = n // self.batch
        losses = torch.zeros((max(nb, 1), 2), dtype=torch.float32, device=self.dev)
        for b in range(nb):
            self.step(desc, labels, perm[b * self.batch:(b + 1) * self.batch], loss=losses[b], ft=ft)
        if nb:
            self.loss.copy_(losses[nb - 1])
        mean = (losses[:nb].double().sum(0) / max(nb, 1)).cpu().numpy()
        self.fm_loss = float(mean[1])
        return float(mean[0])

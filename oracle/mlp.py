"""ORACLE (test infrastructure only): the pair-energy network in FP64 numpy.

Paper section 2: a fully connected feed-forward network g_NN_U maps the pair
configuration to the pair energy; supplementary section 6 takes forces and
torques from its gradient.  The workload fixes the network: 7 inputs (the
separation in body i's frame and the relative quaternion), four hidden
layers of width 128 with SiLU, one linear output.  Weights of layer l are
W_l (out x in) and b_l; the flat parameter vector stores, layer by layer,
W_l row-major then b_l.

Normalisation: the network sees u' = (u - in_shift) * in_scale and its raw
output e' becomes E = e' * out_scale + out_shift.  The training loss is the
mean squared error in normalised units, mean((e' - y')^2) with
y' = (y - out_shift) / out_scale.  Adam follows Kingma and Ba (ICLR 2015).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import frames

DIMS = (7, 128, 128, 128, 128, 1)


@dataclass
class Norm:
    in_shift: np.ndarray = field(default_factory=lambda: np.zeros(7))
    in_scale: np.ndarray = field(default_factory=lambda: np.ones(7))
    out_shift: float = 0.0
    out_scale: float = 1.0

    def as_array(self) -> np.ndarray:
        """16 numbers: in_shift[7], in_scale[7], out_shift, out_scale."""
        return np.concatenate([self.in_shift, self.in_scale, [self.out_shift, self.out_scale]])


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 value (ties to even), as FP64.

    BF16 keeps the upper 16 bits of an FP32 number; rounding adds half of
    the dropped part, with ties resolved toward an even kept part.
    """
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_network(params: np.ndarray, dims=DIMS) -> np.ndarray:
    """The network the BF16 kernels implement: the three hidden-to-hidden
    weight matrices rounded to BF16, every other parameter kept in FP32."""
    layers = unpack(np.asarray(params, dtype=np.float32).astype(np.float64), dims)
    out = []
    for li, (W, b) in enumerate(layers):
        out.append((round_bf16(W) if 0 < li < len(layers) - 1 else W, b))
    return pack(out)


def unpack(params: np.ndarray, dims=DIMS) -> list[tuple[np.ndarray, np.ndarray]]:
    params = np.asarray(params, dtype=np.float64)
    layers, o = [], 0
    for fi, fo in zip(dims[:-1], dims[1:]):
        W = params[o:o + fo * fi].reshape(fo, fi)
        o += fo * fi
        b = params[o:o + fo]
        o += fo
        layers.append((W, b))
    assert o == params.size, "parameter vector does not match the layer sizes"
    return layers


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def _sigmoid(z):
    with np.errstate(over="ignore"):
        return 1.0 / (1.0 + np.exp(-z))


def act(z, kind="silu"):
    if kind == "identity":
        return z
    return z * _sigmoid(z)


def act_grad(z, kind="silu"):
    if kind == "identity":
        return np.ones_like(z)
    s = _sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def _forward(params, u, norm, kind, dims):
    norm = norm or Norm()
    layers = unpack(params, dims)
    a = (np.asarray(u, dtype=np.float64) - norm.in_shift) * norm.in_scale
    acts, zs = [a], []
    for W, b in layers[:-1]:
        z = a @ W.T + b
        zs.append(z)
        a = act(z, kind)
        acts.append(a)
    W, b = layers[-1]
    e = (a @ W.T + b)[:, 0]
    return e, acts, zs, layers, norm


def forward(params, u, norm: Norm | None = None, kind="silu", dims=DIMS) -> np.ndarray:
    """Pair energies E (P,) for descriptors u (P, 7)."""
    e, _, _, _, norm = _forward(params, u, norm, kind, dims)
    return e * norm.out_scale + norm.out_shift


def _backward(delta_out, acts, zs, layers, kind):
    """Back-propagate dX/de' (P,) through the layers.

    Returns the gradient with respect to the normalised input and the list of
    (dW_l, db_l) summed over the rows.
    """
    grads = []
    W, b = layers[-1]
    grads.append((delta_out[:, None].T @ acts[-1], np.array([delta_out.sum()])))
    g = delta_out[:, None] * W                      # dX/da_4, (P, 128)
    for li in range(len(layers) - 2, -1, -1):
        delta = g * act_grad(zs[li], kind)          # dX/dz_l
        Wl, _ = layers[li]
        grads.append((delta.T @ acts[li], delta.sum(axis=0)))
        g = delta @ Wl                              # dX/da_{l-1}
    grads.reverse()
    return g, grads


def input_grad(params, u, norm: Norm | None = None, kind="silu", dims=DIMS):
    """(E, dE/du) with dE/du of shape (P, 7), by reverse-mode chain rule."""
    e, acts, zs, layers, norm = _forward(params, u, norm, kind, dims)
    g, _ = _backward(np.ones_like(e), acts, zs, layers, kind)
    return e * norm.out_scale + norm.out_shift, g * norm.in_scale * norm.out_scale


def loss_and_grad(params, u, y, norm: Norm | None = None, kind="silu", dims=DIMS):
    """Training loss mean((e' - y')^2) and its gradient w.r.t. the parameters."""
    e, acts, zs, layers, norm = _forward(params, u, norm, kind, dims)
    yn = (np.asarray(y, dtype=np.float64) - norm.out_shift) / norm.out_scale
    r = e - yn
    loss = float(np.mean(r * r))
    _, grads = _backward(2.0 * r / len(r), acts, zs, layers, kind)
    return loss, pack(grads)


def adam_step(params, m, v, t, g, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; t is the 1-based index of this update.  Returns new
    (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


def act_grad2(z, kind="silu"):
    """Second derivative of the activation."""
    if kind == "identity":
        return np.zeros_like(z)
    s = _sigmoid(z)
    return s * (1.0 - s) * (2.0 + z * (1.0 - 2.0 * s))


def fm_loss_and_grad(params, u, y, ft, lam_f, lam_t, norm: Norm | None = None, kind="silu", dims=DIMS):
    """Energy loss plus force/torque matching, and the exact parameter
    gradient.

    loss = mean((e' - y')^2) + lam_f mean |F_j - F_j*|^2 + lam_t mean
    |tau_j - tau_j*|^2, with F_j, tau_j from the network's input gradient
    (frames.forces_from_grad) and ft = (F_j*, tau_j*) (P, 6) the labels, in
    physical units.
    Returns (energy term, force/torque term, gradient).

    The force/torque term depends on the parameters through g = dE/du; its
    gradient is sum_b v_b . dg_b/dtheta with v_b = dL/dg_b, i.e. the
    parameter gradient of the directional derivative of E along v_b.  That
    derivative is carried forward (tangents z_l', a_l' of every layer) and
    then differentiated in reverse through both the tangent and the primal
    chains (second derivative of the activation where they meet).
    """
    norm = norm or Norm()
    u = np.asarray(u, np.float64)
    P = len(u)
    e_loss, g_e = loss_and_grad(params, u, y, norm, kind, dims)
    e, acts, zs, layers, norm = _forward(params, u, norm, kind, dims)
    gn, _ = _backward(np.ones_like(e), acts, zs, layers, kind)
    g = gn * norm.in_scale * norm.out_scale                     # dE/du, physical
    fr = frames.forces_from_grad(u, g)
    F, tau = fr[:, :3], fr[:, 6:9]
    dF, dT = F - ft[:, :3], tau - ft[:, 3:6]
    fm_loss = float(lam_f * np.mean((dF * dF).sum(1)) + lam_t * np.mean((dT * dT).sum(1)))
    wF, wT = 2.0 * lam_f * dF / P, 2.0 * lam_t * dT / P
    # v = dL/dg through F_j = -g_d, tau_j = -(w g_v - g_w v + v x g_v) / 2
    wq, vq = u[:, 3:4], u[:, 4:7]
    v = np.zeros_like(u)
    v[:, :3] = -wF
    v[:, 3] = 0.5 * (wT * vq).sum(1)
    v[:, 4:7] = -0.5 * (wq * wT + np.cross(wT, vq))
    # v . g = out_scale * (v * in_scale) . g_n: tangent along vt in normalised
    # input units, then scaled by out_scale
    vt = v * norm.in_scale
    adot, zdot = [vt], [None]          # tangents a_l', z_l' (layer 0: the input)
    for li, (W, _) in enumerate(layers[:-1]):
        zdot.append(adot[-1] @ W.T)
        adot.append(act_grad(zs[li], kind) * zdot[-1])
    grads = [None] * len(layers)
    W5, _ = layers[-1]
    grads[-1] = (norm.out_scale * adot[-1].sum(0)[None, :], np.zeros(1))
    abar = np.broadcast_to(W5, (P, W5.shape[1])) * norm.out_scale   # adjoint of a_4'
    pbar = np.zeros_like(abar)                                      # adjoint of a_4 (primal)
    for li in range(len(layers) - 2, -1, -1):
        W, _ = layers[li]
        z = zs[li]
        zdbar = abar * act_grad(z, kind)                            # adjoint of z_l'
        zbar = abar * zdot[li + 1] * act_grad2(z, kind) + pbar * act_grad(z, kind)
        dW = zdbar.T @ adot[li] + zbar.T @ acts[li]
        db = zbar.sum(0)
        grads[li] = (dW, db)
        abar = zdbar @ W
        pbar = zbar @ W
    return e_loss, fm_loss, g_e + pack(grads)

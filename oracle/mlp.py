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

"""FP64 reference of the learned collision closure (test infrastructure only).

Only tests/, the smoke check and bench.py's CPU-baseline leg use this
module; it shares no code with the GPU library.

The closure (an addition of this library; nothing in the paper): a
19 -> 64 -> 64 -> 19 perceptron with tanh-form GELU activations maps the
standardized non-equilibrium part of a voxel per unit density,
g = (f - f^eq(rho, u)) / rho, to an estimate y of the regularized
non-equilibrium part per unit density, f1/rho (the Hermite projection of
the regularized collision).  The
estimate is projected onto the second-order Hermite space, the space the
regularized operator's f1 lives in,

    P(y)_i = w_i / (2 c_s^4) Q_i : sum_j Q_j y_j,   Q_i = c_i c_i - c_s^2 I,

so that it carries no mass, no momentum and no non-hydrodynamic (ghost)
content, and the post-collision state is f* = f^eq + (1 - 1/tau) rho P(y).
(The network thus supplies the non-equilibrium stress; a projection that
only removed mass and momentum let ghost content through, which near
tau = 1/2 is relaxed with a factor close to -1 and grew in closed loop.)  A voxel
falls back to the regularized operator if any standardized input exceeds 8
in magnitude, if any output population is negative, or -- the regularized
operator acting as judge of the closure's error -- if
|P(y) - f1/rho|_2^2 > judge^2 (|f1/rho|_2^2 + |out_std|_2^2) (judge = 0.01
by default; 0 disables the test; the floor, the typical training-target
size, lets voxels near equilibrium, whose f1 is almost zero, keep the
network's update when its deviation is small in absolute terms).  Near tau = 1/2 the non-equilibrium part is relaxed by a factor
close to -1, and a closure that overshoots the regularized stress by more
than about 1/(1 - 1/tau) - 1 (1.5% at tau = 0.5038) makes that factor
exceed 1 in magnitude; the judge keeps every accepted update inside it.  Training minimizes the
mean squared error between P(y) and f1/rho, divided by the mean target
variance (mean of out_std^2) so that the loss is scale free, with Adam.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import oracle as _orc

K_GELU = math.sqrt(2.0 / math.pi)
A_GELU = 0.044715
HIDDEN = 64
Q = 19
FALLBACK_LIMIT = 8.0
JUDGE = 0.01
JUDGE_FLOOR = 1.0


def gelu(x):
    """GELU, tanh form: 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3)))."""
    return 0.5 * x * (1.0 + np.tanh(K_GELU * (x + A_GELU * x ** 3)))


def gelu_grad(x):
    t = np.tanh(K_GELU * (x + A_GELU * x ** 3))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * K_GELU * (1.0 + 3.0 * A_GELU * x * x)


def lattice():
    c, w, _ = _orc.lattice()
    return c.astype(np.float64), w


def hermite_tensors():
    """Q_i = c_i c_i - c_s^2 I for every direction, shape (19, 3, 3)."""
    c, _ = lattice()
    return np.einsum("ia,ib->iab", c, c) - np.eye(3)[None] / 3.0


def projection_matrix():
    """M with P(y) = y M^T for row vectors y: M_ij = w_i (Q_i : Q_j) / (2 c_s^4)."""
    _, w = lattice()
    Qt = hermite_tensors()
    return 4.5 * w[:, None] * np.einsum("iab,jab->ij", Qt, Qt)


def project(y):
    """Second-order Hermite projection of y (..., 19)."""
    _, w = lattice()
    Qt = hermite_tensors()
    pi = np.einsum("...j,jab->...ab", np.asarray(y, np.float64), Qt)
    return 4.5 * w * np.einsum("iab,...ab->...i", Qt, pi)


@dataclass
class Params:
    W1: np.ndarray  # (19, 64)
    b1: np.ndarray  # (64,)
    W2: np.ndarray  # (64, 64)
    b2: np.ndarray
    W3: np.ndarray  # (64, 19)
    b3: np.ndarray  # (19,)
    in_mean: np.ndarray
    in_std: np.ndarray
    out_mean: np.ndarray
    out_std: np.ndarray

    TRAINED = ("W1", "b1", "W2", "b2", "W3", "b3")

    def trained(self):
        return [getattr(self, k) for k in self.TRAINED]

    def copy(self):
        return Params(*[np.array(getattr(self, f), np.float64, copy=True) for f in self.__dataclass_fields__])

    def bf16_rounded(self):
        """Trained weights rounded to bfloat16 (nearest-even), as the GPU
        forward uses them; standardization stays FP64."""
        p = self.copy()
        for k in self.TRAINED:
            setattr(p, k, bf16_round(getattr(p, k)))
        return p


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32).view(np.float32)).astype(np.float64)


def forward(p: Params, g, cache: bool = False):
    x = (np.asarray(g, np.float64) - p.in_mean) / p.in_std
    z1 = x @ p.W1 + p.b1
    h1 = gelu(z1)
    z2 = h1 @ p.W2 + p.b2
    h2 = gelu(z2)
    yt = h2 @ p.W3 + p.b3
    y = yt * p.out_std + p.out_mean
    if cache:
        return y, (x, z1, h1, z2, h2)
    return y


def loss(p: Params, g, target):
    d = project(forward(p, g)) - target
    return float(np.mean(d * d) / np.mean(p.out_std ** 2))


def backward(p: Params, g, target):
    """Gradients of loss() with respect to W1, b1, W2, b2, W3, b3."""
    y, (x, z1, h1, z2, h2) = forward(p, g, cache=True)
    n = y.shape[0]
    dP = 2.0 * (project(y) - target) / (n * Q * np.mean(p.out_std ** 2))
    dy = dP @ projection_matrix()
    dyt = dy * p.out_std
    gW3 = h2.T @ dyt
    gb3 = dyt.sum(0)
    dz2 = (dyt @ p.W3.T) * gelu_grad(z2)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ p.W2.T) * gelu_grad(z1)
    gW1 = x.T @ dz1
    gb1 = dz1.sum(0)
    return [gW1, gb1, gW2, gb2, gW3, gb3]


@dataclass
class Adam:
    lr: float = 1e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8

    def step(self, params, grads, m, v, t):
        """One Adam update (t counts from 1); updates params, m, v in place."""
        for k, (w, gr) in enumerate(zip(params, grads)):
            m[k] = self.beta1 * m[k] + (1 - self.beta1) * gr
            v[k] = self.beta2 * v[k] + (1 - self.beta2) * gr * gr
            mh = m[k] / (1 - self.beta1 ** t)
            vh = v[k] / (1 - self.beta2 ** t)
            w -= self.lr * mh / (np.sqrt(vh) + self.eps)


def regularized_target(f):
    """f1 / rho of the regularized operator for populations f (..., 19)."""
    f = np.asarray(f, np.float64).reshape(-1, Q)
    out = np.zeros_like(f)
    for k in range(f.shape[0]):
        rho, u = _orc.moments(f[k])
        feq = _orc.equilibrium(rho, u)
        out[k] = _orc.f1_projection(f[k], feq) / rho
    return out


def closure_inputs(f):
    """g = (f - f^eq(rho, u)) / rho for populations f (N, 19)."""
    f = np.asarray(f, np.float64).reshape(-1, Q)
    out = np.zeros_like(f)
    for k in range(f.shape[0]):
        rho, u = _orc.moments(f[k])
        out[k] = (f[k] - _orc.equilibrium(rho, u)) / rho
    return out


def collide(p: Params, f, tau, y_override=None, judge: float = JUDGE):
    """Post-collision populations of the closure for f (N, 19); returns
    (f*, fell_back (N,) bool).  y_override replaces the network output
    (used to check the assembly against the regularized operator)."""
    f = np.asarray(f, np.float64).reshape(-1, Q)
    g = closure_inputs(f)
    y = forward(p, g) if y_override is None else np.asarray(y_override, np.float64)
    py = project(y)
    t = regularized_target(f)
    out = np.zeros_like(f)
    fell = np.zeros(f.shape[0], bool)
    x = (g - p.in_mean) / p.in_std
    for k in range(f.shape[0]):
        rho, u = _orc.moments(f[k])
        feq = _orc.equilibrium(rho, u)
        fs = feq + (1.0 - 1.0 / tau) * rho * py[k]
        floor2 = (JUDGE_FLOOR ** 2) * np.sum(p.out_std ** 2)
        off = judge > 0 and np.sum((py[k] - t[k]) ** 2) > judge * judge * (np.sum(t[k] ** 2) + floor2)
        if np.any(np.abs(x[k]) > FALLBACK_LIMIT) or np.any(fs < 0) or off:
            fs = _orc.collide_regularized(f[k], tau)
            fell[k] = True
        out[k] = fs
    return out, fell

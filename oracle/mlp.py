"""FP64 reference of the learned macro-step network: forward, manual backprop, MSE, Adam.

Test infrastructure (see ``oracle/__init__``).  The network is not part of the paper; it is
the per-element surrogate of M explicit substeps of the propagation problem (Sec. 3.2).

Network: x (80) -> Linear(256) -> GELU -> Linear(256) -> GELU -> Linear(256) -> GELU ->
Linear(20).  GELU is the erf form, gelu(z) = z Phi(z) with Phi the standard normal CDF.
Loss: mean squared error over batch and outputs.  Optimiser: Adam with bias correction.

Flat parameter order: W1 [256,80], b1 [256], W2 [256,256], b2, W3 [256,256], b3, W4 [20,256],
b4 [20]  (W[i] maps layer input to output as y = x W^T + b).

Input of one element T (2D, P^k, d = 2): [c_T, c_N0, c_N1, c_N2] with N_j the neighbour across
local facet j (opposite vertex j), each flattened [d, Np], all divided by the scale s and
multiplied by the element's orientation sign sigma = sign of the x component of v_1 - v_0.
The point reflection x -> 2c - x maps a solution of w_t + div(w (x) w) = 0 to the solution
-w(2c - x), maps each element's coefficients to minus themselves in the reflected element's
frame, and swaps the two triangles of a split square (their first edges point in opposite x
directions), so one network serves both.  The network output y_T is the remainder of the
macro-step beyond forward Euler over tau = M dt, in units of s^3 tau^2 / h:
w_T <- w_T + tau r(w)_T + sigma_T (s^3 tau^2 / h) y_T.
"""
import numpy as np
from scipy.special import erf

SIZES = [(256, 80), (256, 256), (256, 256), (20, 256)]


def n_params():
    return sum(o * i + o for o, i in SIZES)


def unflatten(p):
    out, off = [], 0
    for o, i in SIZES:
        W = p[off:off + o * i].reshape(o, i)
        off += o * i
        b = p[off:off + o]
        off += o
        out.append((W, b))
    return out


def init_params(seed=0):
    """He-style init: W ~ N(0, 2/fan_in) (last layer 1/fan_in), b = 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for li, (o, i) in enumerate(SIZES):
        sd = np.sqrt((1.0 if li == len(SIZES) - 1 else 2.0) / i)
        parts.append(rng.normal(0.0, sd, size=o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(p, x, keep=False):
    """y = net(x) for x [B, 80]; with keep=True also the pre-activations and activations."""
    layers = unflatten(p)
    h = x
    zs, hs = [], [x]
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        if li < len(layers) - 1:
            zs.append(z)
            h = gelu(z)
            hs.append(h)
        else:
            h = z
    return (h, zs, hs) if keep else h


def loss_and_grad(p, x, t):
    """MSE loss and its gradient with respect to the flat parameters (manual backprop)."""
    layers = unflatten(p)
    y, zs, hs = forward(p, x, keep=True)
    B, O = y.shape
    loss = np.mean((y - t) ** 2)
    dy = 2.0 * (y - t) / (B * O)
    grads = []
    d = dy
    for li in range(len(layers) - 1, -1, -1):
        W, b = layers[li]
        gW = d.T @ hs[li]
        gb = d.sum(axis=0)
        grads.append((gW, gb))
        if li > 0:
            d = (d @ W) * gelu_grad(zs[li - 1])
    grads.reverse()
    return loss, np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


class Adam:
    """Adam with bias correction (beta1 = 0.9, beta2 = 0.999, eps = 1e-8)."""

    def __init__(self, n, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.b1, self.b2, self.eps = b1, b2, eps

    def step(self, p, g, lr):
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - lr * mh / (np.sqrt(vh) + self.eps)


def features(w, nbr, sign, scale, elems):
    """Network inputs of elements `elems` from the state w [E, d, Np] (see module docstring)."""
    parts = [w[elems]] + [w[nbr[elems, j]] for j in range(nbr.shape[1])]
    x = np.concatenate([q.reshape(len(elems), -1) for q in parts], axis=1)
    return x * (sign[elems] / scale)[:, None]

"""FP64 reference of the learned closure network (TEST INFRASTRUCTURE ONLY).

The closure is not part of arXiv:2211.06142: it is a small per-parcel network
that corrects the coarse-grained drag and cohesion.  Definitions used here:

  features   x = [n, |u - v|, Re, k, mean delta/R*, contact count]   (6)
  normalise  xh = (x - mu) / sigma
  network    z1 = xh W1 + b1,  h1 = gelu(z1)          6 -> 64
             z2 = h1 W2 + b2,  h2 = gelu(z2)         64 -> 64
             z3 = h2 W3 + b3,  h3 = gelu(z3)         64 -> 64
             y  = h3 W4 + b4                         64 -> 2
  gelu(s)  = s Phi(s) = 0.5 s (1 + erf(s / sqrt 2))  (exact form, not tanh)
  factors  c = exp(clip(y, -ln 2, ln 2)): c_drag multiplies the drag force of
           the particle (eq 8), c_coh scales the surface energy of a pair as
           gamma sqrt(c_i c_j)
  loss     L = mean over the batch and both outputs of (y - t)^2, t = log target
  update   Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction

Flat parameter vector (8898 values, row-major W[k][m] with k the input):
  W1 6x64 | b1 64 | W2 64x64 | b2 64 | W3 64x64 | b3 64 | W4 64x2 | b4 2
Everything is plain numpy in float64; a matmul is a library primitive.
"""
import math

import numpy as np
from scipy.special import erf

SIZES = (6, 64, 64, 64, 2)
N_PARAMS = sum(SIZES[i] * SIZES[i + 1] + SIZES[i + 1] for i in range(4))
LN2 = math.log(2.0)
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


def unpack(p):
    """Views (W, b) per layer of the flat parameter vector."""
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (N_PARAMS,)
    out, o = [], 0
    for i in range(4):
        k, m = SIZES[i], SIZES[i + 1]
        W = p[o:o + k * m].reshape(k, m)
        o += k * m
        b = p[o:o + m]
        o += m
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def init_params(seed, scale=1.0):
    """He-style normal initialisation, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    layers = []
    for i in range(4):
        k, m = SIZES[i], SIZES[i + 1]
        layers.append((rng.normal(0.0, scale * math.sqrt(2.0 / k), (k, m)), np.zeros(m)))
    return pack(layers)


def gelu(s):
    return 0.5 * s * (1.0 + erf(s / math.sqrt(2.0)))


def gelu_grad(s):
    """d gelu / ds = Phi(s) + s phi(s)."""
    return 0.5 * (1.0 + erf(s / math.sqrt(2.0))) + s * np.exp(-0.5 * s * s) / math.sqrt(2.0 * math.pi)


def normalise(x, mu, sigma):
    return (np.asarray(x, np.float64) - np.asarray(mu, np.float64)) / np.asarray(sigma, np.float64)


def forward(p, xh, keep=False):
    """y (B x 2) for normalised inputs xh (B x 6); keep=True also returns the
    pre-activations and activations for the backward pass."""
    layers = unpack(p)
    h = np.asarray(xh, np.float64)
    hs, zs = [h], []
    for i, (W, b) in enumerate(layers):
        z = h @ W + b
        zs.append(z)
        h = gelu(z) if i < 3 else z
        hs.append(h)
    return (h, zs, hs) if keep else h


def factors(y):
    """closure factors (c_drag, c_coh) from the network output"""
    return np.exp(np.clip(y, -LN2, LN2))


def loss(p, xh, t):
    y = forward(p, xh)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def grad(p, xh, t):
    """(loss, dL/dp) by the chain rule, layer by layer from the output."""
    y, zs, hs = forward(p, xh, keep=True)
    t = np.asarray(t, np.float64)
    B = y.shape[0]
    g = 2.0 * (y - t) / (B * y.shape[1])        # dL/dy
    layers = unpack(p)
    grads = [None] * 4
    for i in range(3, -1, -1):
        W, _ = layers[i]
        dW = hs[i].T @ g
        db = g.sum(axis=0)
        grads[i] = (dW, db)
        if i > 0:
            g = (g @ W.T) * gelu_grad(zs[i - 1])
    return float(np.mean((y - t) ** 2)), pack(grads)


def adam_step(p, g, m, v, t, lr):
    """One Adam update (step count t >= 1); returns new (p, m, v)."""
    m = ADAM_B1 * m + (1.0 - ADAM_B1) * g
    v = ADAM_B2 * v + (1.0 - ADAM_B2) * g * g
    mh = m / (1.0 - ADAM_B1 ** t)
    vh = v / (1.0 - ADAM_B2 ** t)
    return p - lr * mh / (np.sqrt(vh) + ADAM_EPS), m, v


def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64: the
    values the BF16 operands of the GPU network hold."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)

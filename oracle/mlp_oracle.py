"""mlp_oracle.py -- plain FP64 reference of the viscosity surrogate MLP.

TEST INFRASTRUCTURE ONLY: the tests and the benchmark's checks use it; the
product path never does.  It shares no code with the GPU kernels.

The network (not part of the paper; the learned part of the viscometer
workflow) maps (phi, d/dx, kT, log shear rate), normalised feature by
feature with a fixed mean and standard deviation, through three hidden
layers of 64 SiLU units to log(eta_eff / eta):

    z1 = x W1 + b1, h1 = silu(z1), ..., y = h3 W4 + b4,  silu(z) = z s(z),

with s the logistic function.  Precision reading (stated, not in any
source): the forward and backward passes use the parameters rounded to
bfloat16 (round to nearest, ties to even) while the Adam update keeps
float32 master copies; activations and sums are plain FP64 here (FP32 with
FP32 accumulation on the GPU).  Gradients are those of the rounded
parameters, applied to the masters unchanged.  The loss is the mean squared
error over the batch.  Adam (Kingma & Ba, ICLR 2015) with bias correction.
"""
import numpy as np

LAYERS = (4, 64, 64, 64, 1)


def split(params, layers=LAYERS):
    """Views W1, b1, W2, b2, ... of the flat parameter vector."""
    out, o = [], 0
    for a, b in zip(layers[:-1], layers[1:]):
        out.append(params[o:o + a * b].reshape(a, b))
        o += a * b
        out.append(params[o:o + b])
        o += b
    assert o == params.size
    return out


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even), returned as
    float32 holding the rounded values."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def normalise(x, norm):
    norm = np.asarray(norm, np.float64)
    return (np.asarray(x, np.float64) - norm[:4]) / norm[4:]


def forward(params, x, norm, keep=False, quantise=True):
    """y [n] for inputs x [n x 4]; keep=True also returns the activations.
    quantise=False takes the parameters as given (FP64), for derivative
    checks."""
    q = bf16_round(params) if quantise else params
    P = split(np.asarray(q, np.float64))
    h = normalise(x, norm)
    acts = [h]
    zs = []
    for layer in range(3):
        W, b = P[2 * layer], P[2 * layer + 1]
        z = h @ W + b
        h = silu(z)
        zs.append(z)
        acts.append(h)
    y = (h @ P[6] + P[7])[:, 0]
    return (y, zs, acts) if keep else y


def loss_and_grad(params, x, t, norm, quantise=True):
    """Mean squared error over the batch and its gradient with respect to
    the (rounded) parameters, as a flat FP64 vector."""
    q = bf16_round(params) if quantise else params
    P = split(np.asarray(q, np.float64))
    y, zs, acts = forward(q, x, norm, keep=True, quantise=False)
    n = y.size
    r = y - np.asarray(t, np.float64)
    loss = float(r @ r / n)
    dy = 2.0 * r / n
    grads = [None] * 8
    grads[6] = acts[3].T @ dy[:, None]
    grads[7] = np.array([dy.sum()])
    dh = dy[:, None] @ P[6].T
    for layer in (2, 1, 0):
        dz = dh * silu_grad(zs[layer])
        grads[2 * layer] = acts[layer].T @ dz
        grads[2 * layer + 1] = dz.sum(axis=0)
        dh = dz @ P[2 * layer].T
    return loss, np.concatenate([g.ravel() for g in grads])


class Adam:
    """Adam with bias correction on float32 master parameters (the update
    itself evaluated in FP64 and stored to float32)."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.p = np.asarray(params, np.float32).copy()
        self.m = np.zeros(self.p.size)
        self.v = np.zeros(self.p.size)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        self.p = (self.p.astype(np.float64) - self.lr * mh / (np.sqrt(vh) + self.eps)).astype(np.float32)
        return self.p

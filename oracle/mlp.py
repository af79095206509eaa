"""FP64 reference of the learned surrogate's network and its training step.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU baseline, never by the product path.

Network (the surrogate that maps the 7 LV-elastance, Windkessel and wall
parameters to one beat of inlet pressure and flow):
    h_0 = x_n                                (7 normalised inputs)
    z_l = h_{l-1} W_l^T + b_l,  h_l = GELU(z_l)      l = 1..4, width 512
    y_n = h_4 W_5^T + b_5                    (512 outputs)
GELU is the exact form x Phi(x) with Phi the standard normal CDF (erf).
Inputs are mapped affinely from the training box [lo, hi] onto [-1, 1];
outputs are standardised per output with the training set's mean and
standard deviation (y = mu + sigma * y_n).

Loss: the mean of the squared errors of the standardised outputs over the
batch and the outputs.  Gradients by reverse-mode differentiation written
out layer by layer.  Update: Adam (Kingma and Ba, 2015) with bias
correction.

Parameter layout (also the device layout of the FP32 master copy): for
l = 1..5, W_l (out x in, row-major) followed by b_l (out).

Pins (tests/test_oracle_mlp.py): gradients against central finite
differences; GELU against its symmetry identity and closed values; Adam's
first step and its constant-gradient closed form; a network with zero
hidden weights reduces to its last bias.
"""
import math

import numpy as np

WIDTH = 512
N_IN = 7
N_OUT = 512
N_HIDDEN = 4


def layer_shapes(n_in=N_IN, width=WIDTH, n_hidden=N_HIDDEN, n_out=N_OUT):
    """(out, in) of each linear layer."""
    dims = [n_in] + [width] * n_hidden + [n_out]
    return [(dims[k + 1], dims[k]) for k in range(len(dims) - 1)]


def n_params(shapes):
    return sum(o * i + o for o, i in shapes)


def unpack(theta, shapes):
    """Views (W_l, b_l) into the flat parameter vector."""
    out, k = [], 0
    for o, i in shapes:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


_erf = np.vectorize(math.erf, otypes=[float])


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    Phi = 0.5 * (1.0 + _erf(z / math.sqrt(2.0)))
    phi = np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
    return Phi + z * phi


def normalise_inputs(x, lo, hi):
    return 2.0 * (np.asarray(x, float) - lo) / (hi - lo) - 1.0


def forward(theta, shapes, xn):
    """Standardised outputs and the pre-activations z_l of the hidden layers."""
    layers = unpack(np.asarray(theta, float), shapes)
    h = np.asarray(xn, float)
    zs, hs = [], [h]
    for W, b in layers[:-1]:
        z = h @ W.T + b
        h = gelu(z)
        zs.append(z)
        hs.append(h)
    W, b = layers[-1]
    return h @ W.T + b, zs, hs


def loss(theta, shapes, xn, tn):
    y, _, _ = forward(theta, shapes, xn)
    return float(np.mean((y - tn) ** 2))


def loss_and_grad(theta, shapes, xn, tn):
    """Loss and its gradient with respect to the flat parameter vector."""
    theta = np.asarray(theta, float)
    layers = unpack(theta, shapes)
    y, zs, hs = forward(theta, shapes, xn)
    m, n = y.shape
    L = float(np.mean((y - tn) ** 2))
    grads = [None] * len(layers)
    dz = 2.0 * (y - tn) / (m * n)                 # dL/dy
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        grads[l] = (dz.T @ hs[l], dz.sum(axis=0))  # dL/dW_l, dL/db_l
        if l > 0:
            dz = (dz @ W) * gelu_grad(zs[l - 1])
    g = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, g


class Adam:
    """Adam with bias correction; the state is (m, v, t)."""

    def __init__(self, n, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps

    def step(self, theta, g):
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mh = self.m / (1.0 - self.b1 ** self.t)
        vh = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mh / (np.sqrt(vh) + self.eps)

"""FP64 reference of the scatter surrogate network (TEST INFRASTRUCTURE ONLY).

The surrogate maps 6 features of an (event, pixel) pair -- in the detector frame of
the event's angle: (bin centre - pixel's lateral projection)/R, pixel depth/R,
pixel's lateral projection/R, cos(angle), sin(angle), (E - 180 keV)/120 keV -- through three
hidden layers of 128 units with the tanh form of GELU to one output, the
logarithm of the once-scattered part of the per-event density (shifted and
floored, see the library header).  Loss: mean squared error.

Parameter vector layout (34049 floats): W1[6][128], b1[128], W2[128][128], b2[128],
W3[128][128], b3[128], w4[128], b4[1]; W[i][o] maps input unit i to output unit o.
"""
import numpy as np

H = 128
NIN = 6
SIZES = [("W1", (NIN, H)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
         ("W3", (H, H)), ("b3", (H,)), ("w4", (H,)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)
C_GELU = np.sqrt(2.0 / np.pi)


def unpack(theta):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(C_GELU * (z + 0.044715 * z ** 3)))


def gelu_prime(z):
    u = C_GELU * (z + 0.044715 * z ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * C_GELU * (1.0 + 3 * 0.044715 * z * z)


def forward(theta, X):
    p = unpack(np.asarray(theta, np.float64))
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    z3 = h2 @ p["W3"] + p["b3"]
    h3 = gelu(z3)
    y = h3 @ p["w4"] + p["b4"][0]
    return y, (X, z1, h1, z2, h2, z3, h3)


def loss_and_grad(theta, X, t):
    """Mean squared error over the batch and its gradient (backpropagation)."""
    y, (X, z1, h1, z2, h2, z3, h3) = forward(theta, X)
    p = unpack(np.asarray(theta, np.float64))
    M = y.size
    r = y - np.asarray(t, np.float64)
    loss = np.mean(r * r)
    dy = 2.0 * r / M
    g = {}
    g["w4"] = h3.T @ dy
    g["b4"] = np.array([dy.sum()])
    dz3 = np.outer(dy, p["w4"]) * gelu_prime(z3)
    g["W3"] = h2.T @ dz3
    g["b3"] = dz3.sum(0)
    dz2 = (dz3 @ p["W3"].T) * gelu_prime(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * gelu_prime(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    grad = np.concatenate([g[name].ravel() for name, _ in SIZES])
    return loss, grad

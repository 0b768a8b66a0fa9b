"""FP64 NumPy reference of the learned-schedule MLP (test infrastructure only).

The library's MLP: x[16] -> z1 = W1 x + b1 -> h1 = silu(z1) -> z2 = W2 h1 + b2
-> h2 = silu(z2) -> y = W3 h2 + b3, with silu(z) = z / (1 + exp(-z)); loss =
mean squared error over all outputs; optimizer Adam (Kingma and Ba, "Adam: a
method for stochastic optimization", ICLR 2015, Algorithm 1 with bias
correction).  Parameters are one flat array in the order W1[64][16], b1[64],
W2[64][64], b2[64], W3[nout][64], b3[nout].

The backward pass is the chain rule written out; tests pin it to central finite
differences of `loss`.
"""
import numpy as np

NIN, NH = 16, 64


def param_count(nout):
    return NH * NIN + NH + NH * NH + NH + nout * NH + nout


def unpack(p, nout):
    o = 0
    W1 = p[o:o + NH * NIN].reshape(NH, NIN); o += NH * NIN
    b1 = p[o:o + NH]; o += NH
    W2 = p[o:o + NH * NH].reshape(NH, NH); o += NH * NH
    b2 = p[o:o + NH]; o += NH
    W3 = p[o:o + nout * NH].reshape(nout, NH); o += nout * NH
    b3 = p[o:o + nout]
    return W1, b1, W2, b2, W3, b3


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, nout, x):
    """Returns y [B, nout] and the pre-activations (z1, z2)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64), nout)
    z1 = x @ W1.T + b1
    h1 = silu(z1)
    z2 = h1 @ W2.T + b2
    h2 = silu(z2)
    return h2 @ W3.T + b3, (z1, z2)


def mse(y, t):
    e = y - t
    return float(np.mean(e * e)), 2.0 * e / e.size


def backward(p, nout, x, cache, dy):
    """Gradient of the loss with respect to the flat parameters, given dy."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64), nout)
    z1, z2 = cache
    h1, h2 = silu(z1), silu(z2)
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dz2 = (dy @ W3) * dsilu(z2)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dz1 = (dz2 @ W2) * dsilu(z1)
    gW1 = dz1.T @ x
    gb1 = dz1.sum(0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])


def loss(p, nout, x, t):
    y, _ = forward(p, nout, x)
    return mse(y, t)[0]


def adam(p, g, m, v, lr, b1, b2, eps, step):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(nout, seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((NIN, NH), (NH, NH), (NH, nout)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        parts.append(rng.uniform(-lim, lim, (fan_out, fan_in)).ravel())
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts)

"""FP64 reference of the learned-closure network (test infrastructure only).

A 25 -> 64 -> 64 -> 2 multilayer perceptron with the tanh approximation of
GELU, its mean-squared-error loss, the gradient of that loss by hand-written
back-propagation, and one Adam update (Kingma & Ba 2015, Algorithm 1).
Parameter layout (flat vector of 5954 values), shared with lbm_oracle.c:
W1[64][25], b1[64], W2[64][64], b2[64], W3[2][64], b3[2].
"""
import numpy as np

N_IN, N_H, N_OUT = 25, 64, 2
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("W3", (N_OUT, N_H)),
          ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)
_K = np.sqrt(2.0 / np.pi)


def unpack(w):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(w[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(_K * (x + 0.044715 * x ** 3)))


def gelu_grad(x):
    u = _K * (x + 0.044715 * x ** 3)
    t = np.tanh(u)
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * _K * (1.0 + 3 * 0.044715 * x * x)


def init_weights(seed=0, scale=1.0):
    """Uniform fan-in initialisation, biases zero."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            lim = scale * np.sqrt(3.0 / shape[1])
            d[name] = rng.uniform(-lim, lim, size=shape)
        else:
            d[name] = np.zeros(shape)
    return pack(d)


def forward(w, X):
    """X: (B, 25) -> outputs (B, 2) and the activations back-propagation needs."""
    p = unpack(w)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = gelu(z2)
    out = h2 @ p["W3"].T + p["b3"]
    return out, (X, z1, h1, z2, h2)


def loss(w, X, Y):
    """L = (1/B) sum_samples sum_outputs (out - y)^2."""
    out, _ = forward(w, X)
    return float(np.sum((out - Y) ** 2) / X.shape[0])


def loss_and_grad(w, X, Y):
    p = unpack(w)
    out, (X, z1, h1, z2, h2) = forward(w, X)
    B = X.shape[0]
    d3 = 2.0 * (out - Y) / B                   # dL/d out
    g = {"W3": d3.T @ h2, "b3": d3.sum(0)}
    d2 = (d3 @ p["W3"]) * gelu_grad(z2)        # dL/d z2
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * gelu_grad(z1)        # dL/d z1
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return float(np.sum((out - Y) ** 2) / B), pack(g)


def adam(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (w, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v

"""FP64 oracle of the troubled-cell gate network (test infrastructure only).

Network 12 -> 64 -> 64 -> 1 with ReLU hidden layers and a sigmoid output
that estimates the probability that a cell is troubled (its CWENOZ nonlinear
weights leave the linear weights).  Training loss: class-weighted binary
cross-entropy; optimiser: Adam.  Parameters use one flat float layout (the
same offsets the device library uses):

    mu[16] isig[16] W1[16][64] b1[64] W2[64][64] b2[64] w3[64] b3 theta pad

Inputs are standardised, x = (f - mu) * isig, with features 12..15 zero.

``emulate_bf16=True`` rounds, to bfloat16 with round-to-nearest-even, exactly
the quantities the device rounds before its matrix-core products (x, W1, the
first hidden layer, W2, and in the backward pass dH2 and dH1); every other
quantity stays FP64 here.  With ``emulate_bf16=False`` the network is plain
FP64 and is pinned by central finite differences.
"""
import numpy as np

N_IN, N_PAD, N_H = 12, 16, 64
OFF = {"mu": 0, "isig": 16, "W1": 32, "b1": 32 + 16 * 64, "W2": 1120, "b2": 1120 + 64 * 64, "w3": 5280,
       "b3": 5344, "theta": 5345}
N_PARAM = 5348
TRAINABLE = np.zeros(N_PARAM, bool)
TRAINABLE[OFF["W1"]:OFF["theta"]] = True


def unpack(p):
    p = np.asarray(p, np.float64)
    return dict(mu=p[0:16], isig=p[16:32], W1=p[32:1056].reshape(16, 64), b1=p[1056:1120],
                W2=p[1120:5216].reshape(64, 64), b2=p[5216:5280], w3=p[5280:5344], b3=p[5344],
                theta=p[5345])


def bf16(x):
    """Round float values to bfloat16 (round to nearest, ties to even)."""
    f = np.asarray(x, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0, mu=None, sigma=None, theta=0.5):
    """He-initialised weights from a seeded generator (training start)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAM)
    p[0:16] = 0.0 if mu is None else np.pad(mu, (0, 16 - len(mu)))
    isig = np.ones(16) if sigma is None else np.pad(1.0 / np.asarray(sigma), (0, 16 - len(sigma)))
    isig[N_IN:] = 0.0
    p[16:32] = isig
    W1 = rng.normal(0, np.sqrt(2.0 / N_IN), (16, 64))
    W1[N_IN:] = 0.0
    p[32:1056] = W1.ravel()
    p[1120:5216] = rng.normal(0, np.sqrt(2.0 / 64), (64, 64)).ravel()
    p[5280:5344] = rng.normal(0, np.sqrt(1.0 / 64), 64)
    p[5345] = theta
    return p


def forward(p, F, emulate_bf16=False):
    q = unpack(p)
    F = np.asarray(F, np.float64)
    x = np.zeros((F.shape[0], 16))
    x[:, :N_IN] = (F[:, :N_IN] - q["mu"][:N_IN]) * q["isig"][:N_IN]
    W1, W2 = q["W1"], q["W2"]
    if emulate_bf16:
        x, W1, W2 = bf16(x), bf16(W1), bf16(W2)
    h1p = x @ W1 + q["b1"]
    h1 = np.maximum(h1p, 0.0)
    h1m = bf16(h1) if emulate_bf16 else h1
    h2p = h1m @ W2 + q["b2"]
    h2 = np.maximum(h2p, 0.0)
    z = h2 @ q["w3"] + q["b3"]
    return z, dict(x=x, W1=W1, W2=W2, h1p=h1p, h1=h1m, h2p=h2p, h2=h2)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss_and_grad(p, F, y, pos_weight, emulate_bf16=False):
    """Mean class-weighted BCE-with-logits and its gradient (flat layout)."""
    q = unpack(p)
    y = np.asarray(y, np.float64)
    B = len(y)
    z, c = forward(p, F, emulate_bf16)
    w = np.where(y > 0.5, pos_weight, 1.0)
    loss = np.mean(w * (np.logaddexp(0.0, -np.abs(z)) + np.maximum(z, 0.0) - z * y))
    dz = w * (sigmoid(z) - y) / B
    g = np.zeros(N_PARAM)
    dh2 = dz[:, None] * q["w3"][None, :] * (c["h2p"] > 0)
    g[OFF["w3"]:OFF["w3"] + 64] = c["h2"].T @ dz
    g[OFF["b3"]] = dz.sum()
    g[OFF["b2"]:OFF["b2"] + 64] = dh2.sum(0)
    dh2m = bf16(dh2) if emulate_bf16 else dh2
    g[OFF["W2"]:OFF["W2"] + 4096] = (c["h1"].T @ dh2m).ravel()
    dh1 = (dh2m @ c["W2"].T) * (c["h1p"] > 0)
    g[OFF["b1"]:OFF["b1"] + 64] = dh1.sum(0)
    dh1m = bf16(dh1) if emulate_bf16 else dh1
    dW1 = c["x"].T @ dh1m
    dW1[N_IN:] = 0.0
    g[OFF["W1"]:OFF["W1"] + 1024] = dW1.ravel()
    return loss, g


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the trainable slots (t counts from 1)."""
    m[:] = np.where(TRAINABLE, b1 * m + (1 - b1) * g, m)
    v[:] = np.where(TRAINABLE, b2 * v + (1 - b2) * g * g, v)
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p[:] = np.where(TRAINABLE, p - lr * mh / (np.sqrt(vh) + eps), p)
    return p

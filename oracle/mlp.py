"""fp64 reference of the selector MLP -- TEST INFRASTRUCTURE ONLY.

Network (16 -> 64 -> 64 -> 16, ReLU on the hidden layers), masked mean squared
error, its gradient by the chain rule, and one Adam step (Kingma & Ba, "Adam: a
method for stochastic optimization", 2015, Algorithm 1 with bias correction).
The flat parameter layout is W1[16][64], b1[64], W2[64][64], b2[64], W3[64][16],
b3[16], row-major with the input index first. Plain numpy in float64.
"""
import numpy as np

N_IN, N_HID, N_OUT = 16, 64, 16
SHAPES = [("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def forward(flat, X):
    """Returns (Y, H1, H2) for inputs X[B, 16]."""
    P = unpack(flat)
    X = np.asarray(X, dtype=np.float64)
    H1 = np.maximum(X @ P["W1"] + P["b1"], 0.0)
    H2 = np.maximum(H1 @ P["W2"] + P["b2"], 0.0)
    Y = H2 @ P["W3"] + P["b3"]
    return Y, H1, H2


def loss(flat, X, T, M):
    """L = sum(M * (Y - T)^2) / sum(M); 0 for an empty mask."""
    Y, _, _ = forward(flat, X)
    M = np.asarray(M, dtype=np.float64)
    s = M.sum()
    return float((M * (Y - np.asarray(T, dtype=np.float64)) ** 2).sum() / s) if s > 0 else 0.0


def gradient(flat, X, T, M):
    """dL/dparams by the chain rule (ReLU derivative 1 where the output is > 0)."""
    P = unpack(flat)
    X = np.asarray(X, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    Y, H1, H2 = forward(flat, X)
    s = M.sum()
    dY = 2.0 * M * (Y - T) / s if s > 0 else np.zeros_like(Y)
    g = {"W3": H2.T @ dY, "b3": dY.sum(axis=0)}
    dZ2 = (dY @ P["W3"].T) * (H2 > 0)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"].T) * (H1 > 0)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return pack(g)


def adam_step(flat, m, v, g, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns (params, m, v)."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return np.asarray(flat, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v

"""NumPy fp64 oracle of the boundary-closure network (test infrastructure only).

The network is the project's learned replacement for NSBC's extrapolation and
far-field step (eqs. nes_2, nes_3): 96 normalised features of a boundary
node's strip -> 64 (tanh) -> 64 (tanh) -> 3 outputs (the correction of the
NSBC vector m_c in the edge-normal frame).  The GPU runs it with BF16 operands
and FP32 accumulation; with ``bf16=True`` this oracle rounds exactly the same
operands to BF16 (round to nearest even) and does everything else in fp64:

  forward   Z1 = Xb W1b^T + b1, H1 = tanh Z1, H1b = bf16(H1)
            Z2 = H1b W2b^T + b2, H2 = tanh Z2, H2b = bf16(H2)
            Y  = H2b W3b^T + b3                      (Wkb = bf16(Wk), Xb = bf16(X))
  loss      L = mean over the batch and the 3 outputs of (Y - T)^2
  backward  dY = 2 (Y - T) / (3 B),  dYb = bf16(dY)
            dW3 = dYb^T H2b,  db3 = sum dY
            dZ2 = (dYb W3b) * (1 - H2b^2),  dZ2b = bf16(dZ2)
            dW2 = dZ2b^T H1b, db2 = sum dZ2
            dZ1 = (dZ2b W2b) * (1 - H1b^2), dZ1b = bf16(dZ1)
            dW1 = dZ1b^T Xb,  db1 = sum dZ1
  Adam      (Kingma & Ba) on fp32 master weights.

With ``bf16=False`` nothing is rounded: the plain fp64 network, which the
tests pin to finite differences and to an independent autograd.
"""
from __future__ import annotations

import numpy as np

IN, HID, OUT = 96, 64, 3
OUT_PAD = 16


def bf16_round(x) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    out = u.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def init_params(seed: int = 0):
    """Xavier-uniform weights, zero biases (fp32 values held in fp64)."""
    rng = np.random.default_rng(seed)

    def xavier(n_out, n_in):
        a = np.sqrt(6.0 / (n_in + n_out))
        return rng.uniform(-a, a, size=(n_out, n_in)).astype(np.float32).astype(np.float64)

    return {"W1": xavier(HID, IN), "b1": np.zeros(HID), "W2": xavier(HID, HID), "b2": np.zeros(HID),
            "W3": xavier(OUT, HID), "b3": np.zeros(OUT)}


def _r(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(p, X, bf16=True):
    """Returns (Y, cache)."""
    Xb = _r(X, bf16)
    W1, W2, W3 = _r(p["W1"], bf16), _r(p["W2"], bf16), _r(p["W3"], bf16)
    Z1 = Xb @ W1.T + p["b1"]
    H1 = np.tanh(Z1)
    H1b = _r(H1, bf16)
    Z2 = H1b @ W2.T + p["b2"]
    H2 = np.tanh(Z2)
    H2b = _r(H2, bf16)
    Y = H2b @ W3.T + p["b3"]
    return Y, {"Xb": Xb, "H1b": H1b, "H2b": H2b, "W1": W1, "W2": W2, "W3": W3}


def loss(p, X, T, bf16=True) -> float:
    Y, _ = forward(p, X, bf16)
    return float(np.mean((Y - T) ** 2))


def loss_and_grads(p, X, T, bf16=True):
    Y, c = forward(p, X, bf16)
    B = X.shape[0]
    L = float(np.mean((Y - T) ** 2))
    dY = 2.0 * (Y - T) / (OUT * B)
    dYb = _r(dY, bf16)
    g = {"W3": dYb.T @ c["H2b"], "b3": dY.sum(0)}
    dZ2 = (dYb @ c["W3"]) * (1.0 - c["H2b"] ** 2)
    dZ2b = _r(dZ2, bf16)
    g["W2"] = dZ2b.T @ c["H1b"]
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2b @ c["W2"]) * (1.0 - c["H1b"] ** 2)
    dZ1b = _r(dZ1, bf16)
    g["W1"] = dZ1b.T @ c["Xb"]
    g["b1"] = dZ1.sum(0)
    return L, g


def adam_init(p):
    return {k: np.zeros_like(v) for k, v in p.items()}, {k: np.zeros_like(v) for k, v in p.items()}


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new params, m, v."""
    p2, m2, v2 = {}, {}, {}
    for k in p:
        m2[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v2[k] = beta2 * v[k] + (1 - beta2) * g[k] ** 2
        mh = m2[k] / (1 - beta1 ** t)
        vh = v2[k] / (1 - beta2 ** t)
        p2[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p2, m2, v2

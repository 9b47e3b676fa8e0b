"""CPU float64 oracle of the learned GENO gate: the small MLP that predicts the
path function chi (Eq. (4)) of a cell from its normalised stencil, its loss,
gradients and Adam update, and the harvest definition (network input and
target) of a cell of a 2-D state.

TEST INFRASTRUCTURE, NOT PRODUCT CODE: only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import this module. It shares no
code with the HIP library or its binding. Written from the definitions:
matrix products are numpy's, everything else is spelled out.

Network (6849 parameters, flat float vector in this order):
  W1[64][40], b1[64], W2[64][64], b2[64], w3[64], b3
  a1 = W1 x + b1, h1 = gelu(a1), a2 = W2 h1 + b2, h2 = gelu(a2),
  z = w3 . h2 + b3 (logit), p = sigmoid(z) (the predicted chi).
gelu(u) = u/2 (1 + tanh(sqrt(2/pi) (u + 0.044715 u^3))) (the tanh form of
the Gaussian error linear unit, used on both sides).
Loss: mean binary cross-entropy of p against the target chi in [0, 1],
  L = mean(softplus(z) - y z).
"""
from __future__ import annotations

import math

import numpy as np

NIN, NHID = 40, 64
NPARAM = NHID * NIN + NHID + NHID * NHID + NHID + NHID + 1   # 6849
_C = math.sqrt(2.0 / math.pi)


def unpack(p):
    p = np.asarray(p, dtype=np.float64)
    assert p.shape == (NPARAM,)
    o = 0
    W1 = p[o:o + NHID * NIN].reshape(NHID, NIN); o += NHID * NIN
    b1 = p[o:o + NHID]; o += NHID
    W2 = p[o:o + NHID * NHID].reshape(NHID, NHID); o += NHID * NHID
    b2 = p[o:o + NHID]; o += NHID
    w3 = p[o:o + NHID]; o += NHID
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]]).astype(np.float64)


def init(seed):
    """He-scaled normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((NHID, NIN)) * math.sqrt(2.0 / NIN)
    W2 = rng.standard_normal((NHID, NHID)) * math.sqrt(2.0 / NHID)
    w3 = rng.standard_normal(NHID) * math.sqrt(1.0 / NHID)
    return pack(W1, np.zeros(NHID), W2, np.zeros(NHID), w3, 0.0)


def gelu(u):
    return 0.5 * u * (1.0 + np.tanh(_C * (u + 0.044715 * u ** 3)))


def gelu_d(u):
    """d gelu / du by the product and chain rules."""
    t = np.tanh(_C * (u + 0.044715 * u ** 3))
    return 0.5 * (1.0 + t) + 0.5 * u * (1.0 - t * t) * _C * (1.0 + 3.0 * 0.044715 * u * u)


def forward(p, X):
    """Logits z and the activations of each layer."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    z = h2 @ w3 + b3
    return z, (X, a1, h1, a2, h2)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def loss(p, X, y):
    z, _ = forward(p, X)
    # softplus(z) - y z, written stably
    sp = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return float(np.mean(sp - np.asarray(y, dtype=np.float64) * z))


def grad(p, X, y):
    """Gradient of the mean loss by back-propagation (flat, in parameter order)."""
    W1, b1, W2, b2, w3, b3 = unpack(p)
    z, (X, a1, h1, a2, h2) = forward(p, X)
    n = X.shape[0]
    dz = (sigmoid(z) - np.asarray(y, dtype=np.float64)) / n
    dw3 = h2.T @ dz
    db3 = dz.sum()
    da2 = np.outer(dz, w3) * gelu_d(a2)
    dW2 = da2.T @ h1
    db2 = da2.sum(axis=0)
    da1 = (da2 @ W2) * gelu_d(a1)
    dW1 = da1.T @ X
    db1 = da1.sum(axis=0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) with bias correction; t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# harvest: network input and target of one cell and direction of a 2-D state
# ---------------------------------------------------------------------------
def _padded(A, bc, direction, ng=2):
    """Ghost layers along one direction: periodic images or the nearest
    interior cell (transmissive; the normal gradient of a ghost is 0 there)."""
    axis = 2 if direction == 0 else 1
    mode = "wrap" if bc == 0 else "edge"
    pad = [(0, 0)] * 3
    pad[axis] = (ng, ng)
    return np.pad(A, pad, mode=mode)


def harvest(W, dW, direction, bc, h, chi=None):
    """Inputs X[ncell, 40] and, if the oracle's chi of the normal step is
    given (oracle.normal_faces), targets y[ncell] for every interior cell.

    Frame: the conserved variables in the face frame of the direction (normal
    momentum second). Per variable q: den = max - min of q over the 5 cells
    j-2..j+2 along the direction + 1e-12 |q_j| + 1e-300; features
    (q_m - q_j)/den, m = -2..2, then h * (dq/dn)_m / den, m = -2..2, each
    clipped to [-64, 64] (gradients of nearly constant data can be large
    relative to den).
    Feature order: variable-major, 10 per variable.
    Target: min over the cell's two face-sides (the left state of its face
    j+1/2, the right state of its face j-1/2) and the four variables of the
    plain-GENO chi."""
    W = np.asarray(W, dtype=np.float64)
    dW = np.asarray(dW, dtype=np.float64)
    nv, ny, nx = W.shape
    perm = [0, 1, 2, 3] if direction == 0 else [0, 2, 1, 3]
    Q = _padded(W[perm], bc, direction)
    Gn = dW[0:4] if direction == 0 else dW[4:8]
    # the normal gradient of transmissive ghosts is zero
    G = _padded(h * Gn[perm], bc, direction)
    if bc != 0:
        if direction == 0:
            G[:, :, :2] = 0.0
            G[:, :, -2:] = 0.0
        else:
            G[:, :2, :] = 0.0
            G[:, -2:, :] = 0.0
    X = np.zeros((ny, nx, 4, 10))
    for v in range(4):
        if direction == 0:
            qs = np.stack([Q[v, :, 2 + m:2 + m + nx] for m in range(-2, 3)])
            gs = np.stack([G[v, :, 2 + m:2 + m + nx] for m in range(-2, 3)])
        else:
            qs = np.stack([Q[v, 2 + m:2 + m + ny, :] for m in range(-2, 3)])
            gs = np.stack([G[v, 2 + m:2 + m + ny, :] for m in range(-2, 3)])
        q0 = qs[2]
        den = (qs.max(axis=0) - qs.min(axis=0)) + 1e-12 * np.abs(q0) + 1e-300
        X[:, :, v, 0:5] = np.moveaxis((qs - q0) / den, 0, -1)
        X[:, :, v, 5:10] = np.moveaxis(gs / den, 0, -1)
    X = np.clip(X, -64.0, 64.0).reshape(ny * nx, 40)
    if chi is None:
        return X, None
    chi = np.asarray(chi)
    if direction == 0:
        # chi[side, var, a = j + 1, b = face index between cells b-1 and b]
        right_face_left = chi[0, :, 1:ny + 1, 1:nx + 1]
        left_face_right = chi[1, :, 1:ny + 1, 0:nx]
    else:
        # chi[side, var, a = face between rows a-1 and a, b = i + 1]
        right_face_left = chi[0, :, 1:ny + 1, 1:nx + 1]
        left_face_right = chi[1, :, 0:ny, 1:nx + 1]
    y = np.minimum(right_face_left.min(axis=0), left_face_right.min(axis=0)).reshape(-1)
    return X, y

"""FP64 reference of the learned column-density surrogate.

TEST INFRASTRUCTURE ONLY: used by the tests and the benchmark's checks, never
by the product path.  Plain numpy, float64 throughout.

The surrogate is not part of the paper's method: it maps the tree's own
coarse data to the columns the method computes.  What it is built from:

* the pyramid of Sect. 3 (a refined cell holds the mean of its 8 children);
* features per target cell (uniform 2^L grid, L >= 8): for each absolute
  level l = 0 .. 8, the 4^3 level-l cells centred on the centre of the
  target's level-(l-1) ancestor A, i.e. indices 2 A - 1 .. 2 A + 2 per axis
  (the ancestor's 2^3 children and a one-cell ring; at l = 0, A = 0 and only
  the root lies inside the box).  Feature l * 64 + sx + 4 sy + 16 sz is
  ln max(n, 1e-10) at offset (sx, sy, sz), zero density outside the box;
  features are then shifted and scaled, f' = (f - in_shift) / in_scale;
* a multilayer perceptron 576 -> W -> W -> Dout with ReLU activations.  The
  features depend on the target's level-7 ancestor only; for a network
  serving leaf level L (8 or 9) a row of outputs holds a block of D for each
  of the 8^(L-8) octs inside that cell, the scaled log near-shell columns
  y = (ln(E + EXT_FLOOR) - out_shift) / out_scale, E the external sum over
  the shells dl = 1..3 (Sect. 3.2, Eqs. 9-10; shared by the 8 leaves of an
  oct).  The rest of the column is the method's, added back exactly:
  N = N_il + N_far + max(exp(y out_scale + out_shift) - EXT_FLOOR, 0), N_il
  the internal + local part, N_far the shells dl >= 4;
* mean squared error over all outputs and Adam (Kingma & Ba 2015,
  Algorithm 1: beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected).

Pinned (tests/test_oracle_surrogate.py) by: hand-counted feature stencils of a
uniform field at corners, a point mass diluted by 8^-(L-l), gradients against
central finite differences, the closed form of Adam's first step, and a
hand-built network.
"""
from __future__ import annotations

import numpy as np

N_LEVELS = 9
STENCIL = 4
N_FEAT = N_LEVELS * STENCIL ** 3  # 576
FLOOR = 1e-10
EXT_FLOOR = 1e17  # cm^-2 added to the external column before the logarithm
ADAM_B1, ADAM_B2, ADAM_EPS = 0.9, 0.999, 1e-8


# ---------------------------------------------------------------- features --
def pyramid(field_zyx: np.ndarray) -> list:
    """Levels 0 .. L of a uniform 2^L grid, index [z, y, x]; level l < L is
    the mean of the 8 level-(l+1) children (Sect. 3)."""
    f = np.asarray(field_zyx, dtype=np.float64)
    levels = [f]
    while levels[0].shape[0] > 1:
        a = levels[0]
        n = a.shape[0] // 2
        levels.insert(0, a.reshape(n, 2, n, 2, n, 2).mean(axis=(1, 3, 5)))
    return levels


def features(levels: list, cells: np.ndarray, in_shift: float = 0.0, in_scale: float = 1.0) -> np.ndarray:
    """Scaled features [n, 576] of the listed leaves (row-major index, x
    fastest) of a uniform grid whose pyramid is `levels`."""
    L = len(levels) - 1
    assert L >= N_LEVELS - 1, "the features need absolute levels 0 .. 8"
    n = 1 << L
    cells = np.asarray(cells, dtype=np.int64)
    x, y, z = cells % n, (cells // n) % n, cells // (n * n)
    out = np.empty((cells.shape[0], N_FEAT), dtype=np.float64)
    for l in range(N_LEVELS):
        nl = 1 << l
        sh = L - l + 1  # ancestor at level l - 1
        Ax, Ay, Az = x >> sh, y >> sh, z >> sh
        for sz in range(STENCIL):
            for sy in range(STENCIL):
                for sx in range(STENCIL):
                    px, py, pz = 2 * Ax - 1 + sx, 2 * Ay - 1 + sy, 2 * Az - 1 + sz
                    inside = (px >= 0) & (px < nl) & (py >= 0) & (py < nl) & (pz >= 0) & (pz < nl)
                    v = np.zeros(cells.shape[0])
                    v[inside] = levels[l][pz[inside], py[inside], px[inside]]
                    out[:, l * 64 + sx + 4 * sy + 16 * sz] = np.log(np.maximum(v, FLOOR))
    return (out - in_shift) / in_scale


# --------------------------------------------------------------------- MLP --
def param_shapes(width: int, D: int) -> list:
    """Parameter blocks in the library's order: W1 [576, W], b1 [W],
    W2 [W, W], b2 [W], W3 [W, D], b3 [D] (row-major, y = x W + b)."""
    return [(N_FEAT, width), (width,), (width, width), (width,), (width, D), (D,)]


def unflatten(flat: np.ndarray, width: int, D: int) -> list:
    out, o = [], 0
    for s in param_shapes(width, D):
        k = int(np.prod(s))
        out.append(np.asarray(flat[o:o + k], dtype=np.float64).reshape(s))
        o += k
    assert o == flat.shape[0]
    return out


def flatten(params: list) -> np.ndarray:
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1) for p in params])


def forward(params: list, X: np.ndarray):
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1 + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2 + b2
    A2 = np.maximum(Z2, 0.0)
    Y = A2 @ W3 + b3
    return Y, (X, Z1, A1, Z2, A2)


def mse(Y: np.ndarray, T: np.ndarray) -> float:
    return float(np.mean((Y - T) ** 2))


def backward(params: list, cache, Y: np.ndarray, T: np.ndarray) -> list:
    """Gradients of mse(Y, T) (mean over all n x D outputs), same order as
    the parameters."""
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, A1, Z2, A2 = cache
    dY = 2.0 * (Y - T) / Y.size
    dW3 = A2.T @ dY
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3.T) * (Z2 > 0)
    dW2 = A1.T @ dZ2
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2.T) * (Z1 > 0)
    dW1 = X.T @ dZ1
    db1 = dZ1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float):
    """One Adam update (t = 1 for the first step); returns new (p, m, v)."""
    m = ADAM_B1 * m + (1 - ADAM_B1) * g
    v = ADAM_B2 * v + (1 - ADAM_B2) * g * g
    mhat = m / (1 - ADAM_B1 ** t)
    vhat = v / (1 - ADAM_B2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + ADAM_EPS), m, v


def targets(E_near: np.ndarray, out_shift: float, out_scale: float) -> np.ndarray:
    """Scaled log near-shell columns (shells dl = 1..3, cm^-2)."""
    return (np.log(E_near + EXT_FLOOR) - out_shift) / out_scale


def columns_from_output(Y: np.ndarray, N_exact: np.ndarray, out_shift: float, out_scale: float) -> np.ndarray:
    """N (cm^-2) from the network outputs (one block of D) and the parts the
    method supplies exactly (internal + local and shells dl >= 4)."""
    return N_exact + np.maximum(np.exp(Y * out_scale + out_shift) - EXT_FLOOR, 0.0)


def block_of(cells: np.ndarray, L: int) -> np.ndarray:
    """Output block of each leaf's oct inside its level-7 ancestor for a
    network of leaf level L: j = jx + s (jy + s jz), s = 2^(L-8), (jx, jy,
    jz) the oct's offset inside the level-7 cell."""
    n = 1 << L
    cells = np.asarray(cells, dtype=np.int64)
    sb = L - 8
    m = (1 << sb) - 1
    ox, oy, oz = (cells % n) >> 1, ((cells // n) % n) >> 1, (cells // (n * n)) >> 1
    return (ox & m) + ((oy & m) << sb) + ((oz & m) << (2 * sb))


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even), returned as float64: the
    storage format of the library's low-precision weights and activations."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def forward_bf16(params: list, X: np.ndarray):
    """Forward pass with the inputs, weights and hidden activations rounded
    to bfloat16 and sums in float64: the arithmetic the matrix-core path
    approximates (its sums are float32)."""
    W1, b1, W2, b2, W3, b3 = params
    Xb = bf16_round(X)
    A1 = bf16_round(np.maximum(Xb @ bf16_round(W1) + b1, 0.0))
    A2 = bf16_round(np.maximum(A1 @ bf16_round(W2) + b2, 0.0))
    return A2 @ bf16_round(W3) + b3


def backward_bf16(params: list, X: np.ndarray, T: np.ndarray) -> list:
    """Gradients of the bfloat16 network (the forward of forward_bf16):
    the loss gradient, the hidden-layer gradients, inputs and weights are
    rounded to bfloat16 where the matrix-core path stores them, bias
    gradients are summed from the unrounded gradients; sums in float64."""
    W1, b1, W2, b2, W3, b3 = params
    W1b, W2b, W3b = bf16_round(W1), bf16_round(W2), bf16_round(W3)
    Xb = bf16_round(X)
    Z1 = Xb @ W1b + b1
    A1 = bf16_round(np.maximum(Z1, 0.0))
    Z2 = A1 @ W2b + b2
    A2 = bf16_round(np.maximum(Z2, 0.0))
    Y = A2 @ W3b + b3
    dY = 2.0 * (Y - T) / Y.size
    dYb = bf16_round(dY)
    dZ2 = (dYb @ W3b.T) * (Z2 > 0)
    dZ2b = bf16_round(dZ2)
    dZ1 = (dZ2b @ W2b.T) * (Z1 > 0)
    dZ1b = bf16_round(dZ1)
    return [Xb.T @ dZ1b, dZ1.sum(axis=0), A1.T @ dZ2b, dZ2.sum(axis=0), A2.T @ dYb, dY.sum(axis=0)]

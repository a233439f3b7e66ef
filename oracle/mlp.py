"""Learned level selector, oracle side (FP64, explicit formulas).

Network 10 -> H -> H -> K with ReLU hidden layers and a softmax output,
trained with softmax cross-entropy and Adam.  Inputs are standardised by a
stored mean and standard deviation.  Parameter layout (flat):
  W1 [H][10], b1 [H], W2 [H][H], b2 [H], W3 [K][H], b3 [K], mean [10], std [10].
Feature definitions (reading of the selector's inputs):
  log rho, u / sqrt(R T_ref), v / sqrt(R T_ref), log(T / T_ref),
  q_x / (p sqrt(R T)), q_y / (p sqrt(R T)), sigma_xx / p, sigma_xy / p,
  log(1 + dx |grad rho| / rho), log10(Kn_loc) with Kn_loc = lambda / dx,
  lambda = (mu / p) sqrt(pi R T / 2), dx = sqrt(|V|).
"""
from __future__ import annotations

import math

import numpy as np

NF = 10


def n_params(K, H=64):
    return H * NF + H + H * H + H + K * H + K + 2 * NF


def unpack(theta, K, H=64):
    o = 0
    out = []
    for shape in ((H, NF), (H,), (H, H), (H,), (K, H), (K,), (NF,), (NF,)):
        n = int(np.prod(shape))
        out.append(np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape))
        o += n
    return out


def forward(theta, X, K, H=64):
    """Returns logits, probabilities and the cache for backward."""
    W1, b1, W2, b2, W3, b3, mu, sd = unpack(theta, K, H)
    Xn = (np.asarray(X, np.float64) - mu) / sd
    z1 = Xn @ W1.T + b1
    a1 = np.maximum(z1, 0.0)
    z2 = a1 @ W2.T + b2
    a2 = np.maximum(z2, 0.0)
    z3 = a2 @ W3.T + b3
    z = z3 - z3.max(axis=1, keepdims=True)
    e = np.exp(z)
    p = e / e.sum(axis=1, keepdims=True)
    return z3, p, (Xn, z1, a1, z2, a2)


def bf16_round(x):
    """Round to bfloat16 (8 significant bits), to nearest with ties to even.
    The value is first taken in FP32, as the inference kernel holds it."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(theta, X, K, H=64):
    """Inference with BF16 operands (reading of the selector's reduced-precision
    inference): the standardised inputs are formed in FP32, then the inputs,
    the three weight matrices and both hidden activations are rounded to
    bfloat16; biases stay FP32; every sum is taken exactly (FP64).  Returns
    logits and probabilities."""
    W1, b1, W2, b2, W3, b3, mu, sd = unpack(theta, K, H)
    X32 = np.asarray(X, np.float32)
    Xn = bf16_round((X32 - mu.astype(np.float32)) / sd.astype(np.float32))
    a1 = bf16_round(np.maximum(Xn @ bf16_round(W1).T + b1, 0.0))
    a2 = bf16_round(np.maximum(a1 @ bf16_round(W2).T + b2, 0.0))
    z3 = a2 @ bf16_round(W3).T + b3
    e = np.exp(z3 - z3.max(axis=1, keepdims=True))
    return z3, e / e.sum(axis=1, keepdims=True)


def loss_and_grad(theta, X, y, K, H=64):
    """Mean softmax cross-entropy and its gradient w.r.t. the trainable parameters
    (the normalisation entries get zero gradient)."""
    W1, b1, W2, b2, W3, b3, mu, sd = unpack(theta, K, H)
    z3, p, (Xn, z1, a1, z2, a2) = forward(theta, X, K, H)
    B = len(y)
    loss = -np.mean(np.log(p[np.arange(B), y]))
    dz3 = p.copy()
    dz3[np.arange(B), y] -= 1.0
    dz3 /= B
    dW3 = dz3.T @ a2
    db3 = dz3.sum(0)
    da2 = dz3 @ W3
    dz2 = da2 * (z2 > 0)
    dW2 = dz2.T @ a1
    db2 = dz2.sum(0)
    da1 = dz2 @ W2
    dz1 = da1 * (z1 > 0)
    dW1 = dz1.T @ Xn
    db1 = dz1.sum(0)
    g = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3, np.zeros(2 * NF)])
    return loss, g, p


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (bias-corrected); the normalisation block is left unchanged."""
    n_train = len(theta) - 2 * NF
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    th = theta.copy()
    th[:n_train] -= lr * mh[:n_train] / (np.sqrt(vh[:n_train]) + eps)
    return th, m, v


def features(rho, u, v, T, qx, qy, sxx, sxy, gradrho, vol, R, T_ref, mu):
    """Ten selector inputs per cell from macroscopic fields (arrays over cells)."""
    p = rho * R * T
    cs = np.sqrt(R * T)
    lam = (mu / p) * np.sqrt(math.pi * R * T / 2.0)
    dx = np.sqrt(vol)
    return np.stack([np.log(rho), u / math.sqrt(R * T_ref), v / math.sqrt(R * T_ref), np.log(T / T_ref),
                     qx / (p * cs), qy / (p * cs), sxx / p, sxy / p,
                     np.log1p(dx * gradrho / rho), np.log10(lam / dx)], axis=1)


def label_from_masks(cell_kappa, level_kappas, level_sizes):
    """Fewest-point catalogue level whose enclosing mask is no coarser than the
    cell's own mask anywhere (the level that satisfies the cell's requirement);
    -1 if none does."""
    out = np.full(len(cell_kappa), -1, np.int64)
    order = np.argsort(np.asarray(level_sizes), kind="stable")
    for c, kc in enumerate(cell_kappa):
        for l in order:
            if np.all(level_kappas[l] <= kc):
                out[c] = l
                break
    return out


def cell_stress(xi, w, g, rho, u, T, R):
    """Deviatoric stress (sigma_xx, sigma_xy) = (P_xx - p, P_xy), P_ab = sum w c_a c_b g."""
    c = xi - u[None, :]
    pxx = np.sum(w * c[:, 0] * c[:, 0] * g)
    pxy = np.sum(w * c[:, 0] * c[:, 1] * g)
    return pxx - rho * R * T, pxy


def cell_gradient(mesh, rho):
    """|grad rho| per cell: per index direction the central difference (one-sided
    next to a boundary, zero without neighbours), mapped through [t_i; t_j]^-1.
    Unstructured meshes: the unlimited least-squares gradient over the face
    neighbours (a boundary face a zero-gradient ghost at the mirror point)."""
    out = np.zeros(mesh.n_cells)
    if getattr(mesh, "kind", "") == "unstructured":
        from .umesh import lsq_gradient
        for c in range(mesh.n_cells):
            nv = [None if nb < 0 else np.array([rho[nb]]) for nb, _, _ in mesh.cell_faces[c]]
            out[c] = float(np.hypot(*lsq_gradient(mesh, c, np.array([rho[c]]), nv)[0]))
        return out
    for c in range(mesh.n_cells):
        s = np.zeros(2)
        for d in range(2):
            lo, hi = mesh.nbr[c, 2 * d], mesh.nbr[c, 2 * d + 1]
            dl = float(np.hypot(*mesh.dnb[c, 2 * d]))
            dh = float(np.hypot(*mesh.dnb[c, 2 * d + 1]))
            if lo >= 0 and hi >= 0:
                s[d] = (rho[hi] - rho[lo]) / (dl + dh)
            elif hi >= 0:
                s[d] = (rho[hi] - rho[c]) / dh
            elif lo >= 0:
                s[d] = (rho[c] - rho[lo]) / dl
        gvec = mesh.G[c] @ s
        out[c] = float(np.hypot(*gvec))
    return out

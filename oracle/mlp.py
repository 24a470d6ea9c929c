"""Oracle for the learned warm start: per-pore features, Fourier labels, the
multilayer perceptron with its hand-derived backward pass, Adam, and the
assembly of the initial guess.

TEST INFRASTRUCTURE ONLY (tests, the entry-point smoke check and the CPU
baseline leg of the benchmark).  Plain FP64 NumPy.  The paper has no learned
component: this follows the warm-start reading stated with the design (an
initial guess for the FGMRES of Section 4, which stays the judge of the
solution).

* ``features``: own radius; offsets (dx, dy) and radii of the 16 nearest
  pores by centre distance, ties broken by pore index, zero padded; the
  Poiseuille inflow k (H^2 - y_c^2) at the centre height (k = 1/H^2, so the
  peak is 1) and its slope -2 k y_c; the distances to the two walls; zeros up
  to 64 entries.  Heights y_c are measured from the channel centre line.
* ``labels``: per velocity component 32 real Fourier coefficients of the
  density on a pore, a_0, a_1..a_15, b_1..b_15, a_16, with the angle theta
  of each node measured at the pore centre:
  a_0 = mean, a_m = (2/N) sum sigma cos(m theta), b_m = (2/N) sum sigma
  sin(m theta) (the discrete Fourier transform of equispaced samples).
* ``mlp_*``: h_l = GELU(W_l h_{l-1} + b_l) for the hidden layers, identity
  after the last; GELU(x) = x Phi(x) with the exact normal CDF (erf form).
  Inputs are standardised as (x - in_mean) * in_scale and targets as
  (t - out_mean) / out_std; the loss is the mean squared error over all
  standardised outputs.
* ``adam``: Adam with bias correction.
* ``assemble_x0``: the truncated series on every pore, a given wall density
  on the wall, and lambda_k, mu_k from the constraint functionals of the
  completion (the rows that close the system): lambda_k = (1/(2 pi r_k))
  sum w_j sigma_j and mu_k = (1/(2 pi r_k^2)) sum w_j (x_j - c_k)_perp .
  sigma_j with v_perp = (v_y, -v_x).
* ``refine``: one exact solve of the wall rows for the wall density (a block
  Gauss-Seidel step) and the scaling of x0 that minimises the residual norm
  along x0, so that the result is never worse than the zero start.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from . import dlp

N_FEAT = 64
N_COEF = 64
N_NEAR = 16
N_MODES = 16


# ----------------------------------------------------------------------------
# Features and labels
# ----------------------------------------------------------------------------

def features(geom, y_lo: float = 0.0, y_hi: float = 1.0) -> np.ndarray:
    """(M, 64) float64 feature rows, one per pore."""
    m = geom.n_pores
    out = np.zeros((m, N_FEAT))
    hh = 0.5 * (y_hi - y_lo)
    kk = 1.0 / (hh * hh)
    for k in range(m):
        d = [((geom.cx[j] - geom.cx[k]) ** 2 + (geom.cy[j] - geom.cy[k]) ** 2, j)
             for j in range(m) if j != k]
        d.sort()
        out[k, 0] = geom.radius[k]
        for q, (_, j) in enumerate(d[:N_NEAR]):
            out[k, 1 + 3 * q] = geom.cx[j] - geom.cx[k]
            out[k, 2 + 3 * q] = geom.cy[j] - geom.cy[k]
            out[k, 3 + 3 * q] = geom.radius[j]
        yc = geom.cy[k] - 0.5 * (y_lo + y_hi)
        out[k, 49] = kk * (hh * hh - yc * yc)
        out[k, 50] = -2.0 * kk * yc
        out[k, 51] = geom.cy[k] - y_lo
        out[k, 52] = y_hi - geom.cy[k]
    return out


def _angles(geom, k):
    sl = slice(int(geom.curve_off[k]), int(geom.curve_off[k + 1]))
    return np.arctan2(geom.y[sl] - geom.cy[k], geom.x[sl] - geom.cx[k]), sl


def labels(geom, sigma: np.ndarray) -> np.ndarray:
    """(M, 64) Fourier coefficients of the density on every pore."""
    nn = geom.n_nodes
    m = geom.n_pores
    out = np.zeros((m, N_COEF))
    for k in range(m):
        th, sl = _angles(geom, k)
        npk = th.shape[0]
        for comp in range(2):
            s = sigma[comp * nn:(comp + 1) * nn][sl]
            base = 32 * comp
            out[k, base] = s.sum() / npk
            for md in range(1, N_MODES):
                out[k, base + md] = 2.0 / npk * (s * np.cos(md * th)).sum()
                out[k, base + 15 + md] = 2.0 / npk * (s * np.sin(md * th)).sum()
            out[k, base + 31] = 2.0 / npk * (s * np.cos(N_MODES * th)).sum()
    return out


def series(coef_comp: np.ndarray, th: np.ndarray) -> np.ndarray:
    """Evaluate a_0 + sum_{m<16} (a_m cos + b_m sin) + a_16 cos(16 theta)."""
    v = np.full(th.shape, coef_comp[0], dtype=np.float64)
    for md in range(1, N_MODES):
        v += coef_comp[md] * np.cos(md * th) + coef_comp[15 + md] * np.sin(md * th)
    v += coef_comp[31] * np.cos(N_MODES * th)
    return v


def assemble_x0(geom, coeffs: np.ndarray, wall_sigma: np.ndarray | None) -> np.ndarray:
    """Initial guess in the unknown layout [sigma_x | sigma_y | (lx, ly, mu)_k]."""
    nn = geom.n_nodes
    m = geom.n_pores
    x0 = np.zeros(geom.n_unknowns)
    for k in range(m):
        th, sl = _angles(geom, k)
        sx = series(np.asarray(coeffs[k, :32], dtype=np.float64), th)
        sy = series(np.asarray(coeffs[k, 32:], dtype=np.float64), th)
        x0[:nn][sl] = sx
        x0[nn:2 * nn][sl] = sy
        w = geom.w[sl]
        px = geom.x[sl] - geom.cx[k]
        py = geom.y[sl] - geom.cy[k]
        r = geom.radius[k]
        x0[2 * nn + 3 * k] = (w * sx).sum() / (2.0 * math.pi * r)
        x0[2 * nn + 3 * k + 1] = (w * sy).sum() / (2.0 * math.pi * r)
        x0[2 * nn + 3 * k + 2] = (w * (py * sx - px * sy)).sum() / (2.0 * math.pi * r * r)
    if wall_sigma is not None:
        ws = slice(int(geom.curve_off[m]), int(geom.curve_off[m + 1]))
        ne = ws.stop - ws.start
        x0[:nn][ws] = wall_sigma[:ne]
        x0[nn:2 * nn][ws] = wall_sigma[ne:2 * ne]
    return x0


def refine(geom, f: np.ndarray, x0: np.ndarray, apply=None, scale=True):
    """Improve an initial guess: solve the wall rows exactly for the wall
    density with every other unknown fixed, then (scale=True) multiply by
    alpha = <f, A x> / <A x, A x>, the minimiser of ||f - alpha A x||.
    ``apply`` computes A x (default: the oracle's full product)."""
    mv = apply if apply is not None else (lambda v: dlp.apply(geom, v))
    nn = geom.n_nodes
    ws = geom.wall_slice
    wi = np.r_[np.arange(ws.start, ws.stop), nn + np.arange(ws.start, ws.stop)]
    x = np.array(x0, dtype=np.float64)
    if wi.size:
        r = f - mv(x)
        aww = dlp.block(geom, wi, wi)
        x[wi] += np.linalg.solve(aww, r[wi])
    if not scale:
        return x, 1.0
    y = mv(x)
    yy = float(y @ y)
    alpha = float(f @ y) / yy if yy > 0 else 0.0
    return alpha * x, alpha


# ----------------------------------------------------------------------------
# Network
# ----------------------------------------------------------------------------

def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def unpack(flat: np.ndarray, widths):
    """Split a flat parameter vector into [(W_l (out x in), b_l)]: per layer
    W stored column-major, then b."""
    layers, o = [], 0
    for l in range(len(widths) - 1):
        nin, nout = widths[l], widths[l + 1]
        w = np.asarray(flat[o:o + nin * nout], dtype=np.float64).reshape(nin, nout).T
        o += nin * nout
        b = np.asarray(flat[o:o + nout], dtype=np.float64)
        o += nout
        layers.append((w, b))
    return layers


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([w.T.reshape(-1), b]) for w, b in layers])


def mlp_forward(layers, x, scaling=None):
    """x: (batch, in) rows.  Returns de-standardised outputs (batch, out)."""
    in_mean, in_scale, out_mean, out_std = _scaling(layers, scaling)
    h = (np.asarray(x, dtype=np.float64) - in_mean) * in_scale
    for l, (w, b) in enumerate(layers):
        z = h @ w.T + b
        h = gelu(z) if l + 1 < len(layers) else z
    return h * out_std + out_mean


def mlp_loss_grad(layers, x, t, scaling=None):
    """Loss (mean squared error of the standardised targets) and its gradient
    with respect to every W_l and b_l, by the chain rule written out."""
    in_mean, in_scale, out_mean, out_std = _scaling(layers, scaling)
    h = [(np.asarray(x, dtype=np.float64) - in_mean) * in_scale]
    zs = []
    for l, (w, b) in enumerate(layers):
        z = h[-1] @ w.T + b
        zs.append(z)
        h.append(gelu(z) if l + 1 < len(layers) else z)
    tt = (np.asarray(t, dtype=np.float64) - out_mean) / out_std
    diff = h[-1] - tt
    count = diff.size
    loss = float((diff * diff).sum() / count)
    dz = 2.0 * diff / count
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        w, _ = layers[l]
        grads[l] = (dz.T @ h[l], dz.sum(axis=0))
        if l > 0:
            dz = (dz @ w) * gelu_grad(zs[l - 1])
    return loss, grads


def _scaling(layers, scaling):
    nin = layers[0][0].shape[1]
    nout = layers[-1][0].shape[0]
    if scaling is None:
        return np.zeros(nin), np.ones(nin), np.zeros(nout), np.ones(nout)
    return tuple(np.asarray(s, dtype=np.float64) for s in scaling)


def fit_scaling(x, t):
    """Row statistics: input mean and 1/std, target mean and std; a column
    with zero spread keeps scale 1."""
    def stats(a, invert):
        mu = a.mean(axis=0)
        sd = a.std(axis=0)
        flat = ~(sd > 1e-12 * (np.abs(mu) + 1e-30)) | (sd < 1e-30)
        sc = np.where(flat, 1.0, 1.0 / np.where(flat, 1.0, sd) if invert else sd)
        return mu, sc
    a, b = stats(np.asarray(x, dtype=np.float64), True)
    c, d = stats(np.asarray(t, dtype=np.float64), False)
    return a, b, c, d


def adam(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v

"""CPU oracle of the learned initial-state veto bound (TEST INFRASTRUCTURE ONLY).

Plain numpy, written from the definitions below; only tests/, the smoke check
and bench.py's CPU baseline may use it.  The paper has no learned component:
the closest passages are the data-driven fit of the PDF-ratio maxima against eta
(appendix A.2) and the adaptive overestimates it names as future work
(section 5).  What is learned here is an upper bound of the initial-state veto
weight, used as the overestimate constant of a cell of (table entry, eta bin,
ln t cell); the shower checks it on every trial and falls back to the analytic
table when it fails, so it stays exact.

Network: 4 -> 64 -> 64 -> 1, ReLU, parameters (FP32 master, 4545 values)
    W1[64][4] b1[64] W2[64][64] b2[64] W3[64] b3
The forward pass rounds the weights and the first hidden layer to bfloat16
(round to nearest even) and accumulates in FP32, as the matrix-core kernels do.

Features of a logged trial (ln t, ln eta, z, entry):
    x = ((ln t - 10)/10, (ln eta + 7)/7, 2 z - 1, (entry - 40)/32)
Target: y = ln W - ln R[entry][eta bin], the log of the plain-mode weight up to
the alpha_s overestimate (<= 0 because R is a strict bound).

Loss: pinball (quantile) loss at tau, mean over the batch.
Calibration: the margin of a cell (entry, eta bin, ln t cell, the cell the
shower takes for a row's scale) is the largest residual y - f of the held-out
rows in the cell plus 2^-6 when the cell holds at least MIN_CAL_CELL of them;
else that of its (entry, eta bin) over all its cells when they hold at least
MIN_CAL_BIN; else that of its entry when the entry holds at least MIN_CAL;
else infinite (the cell keeps the analytic bound).
Table: R_theta[e][b][k] = min(R[e][b], up6(R[e][b] exp(v))), v = delta_ebk +
max f clipped to [-20, 0],
with f over the probe points of the cell and up6 rounding up to a 7-bit
mantissa (a relative grid of at most 2^-6).

Parity of each function is pinned by the tests (finite differences, closed
forms); the learned shower itself is pinned through the first-emission
distribution and the forced-fallback identity.
"""
from __future__ import annotations

import math

import numpy as np

H = 64
NPARAM = H * 4 + H + H * H + H + H + 1
OFF_W1, OFF_B1 = 0, H * 4
OFF_W2 = OFF_B1 + H
OFF_B2 = OFF_W2 + H * H
OFF_W3 = OFF_B2 + H
OFF_B3 = OFF_W3 + H
assert OFF_B3 + 1 == NPARAM == 4545

NENT_IS, IS0, NB, NTB = 64, 8, 48, 8
LNETA0 = -13.815510557964274  # ln(1e-6): eta bins uniform in ln eta on [1e-6, 1)
DLE = -LNETA0 / NB
MIN_CAL = 2000
MIN_CAL_BIN = 200
MIN_CAL_CELL = 200
V_MIN = -20.0  # the learned bound is at least e^-20 of the analytic one
CAL_MARGIN = 2.0 ** -6
STREAM_MLP = 4
# probe points of a cell: 3 ln t values, 2 ln eta values, 8 z values
NPT, NPE, NPZ = 3, 2, 8
NPROBE = NPT * NPE * NPZ


def bf16(a):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).reshape(a.shape)


def unpack(theta):
    t = np.asarray(theta)
    return (t[OFF_W1:OFF_B1].reshape(H, 4), t[OFF_B1:OFF_W2], t[OFF_W2:OFF_B2].reshape(H, H),
            t[OFF_B2:OFF_W3], t[OFF_W3:OFF_B3], t[OFF_B3])


def init_params(seed: int):
    """He-uniform weights from Philox4x32-10 (key (seed, stream 4), counter
    (p // 4, 0, 0, 0), word p % 4, u = (word + 0.5) / 2^32), zero biases."""
    from oracle.pyoracle import philox4x32
    theta = np.zeros(NPARAM, dtype=np.float32)
    fan = np.zeros(NPARAM)
    fan[OFF_W1:OFF_B1] = 4
    fan[OFF_W2:OFF_B2] = H
    fan[OFF_W3:OFF_B3] = H
    key = (seed & 0xFFFFFFFF, ((seed >> 32) & 0xFFFFFFFF) ^ STREAM_MLP)
    for blk in range((NPARAM + 3) // 4):
        w = philox4x32((blk, 0, 0, 0), key)
        for j in range(4):
            p = 4 * blk + j
            if p >= NPARAM or fan[p] == 0:
                continue
            u = (w[j] + 0.5) / 4294967296.0
            theta[p] = np.float32((2.0 * u - 1.0) * math.sqrt(6.0 / fan[p]))
    return theta


def eta_bin_of_ln(lne):
    b = np.floor((np.asarray(lne, dtype=np.float64) - LNETA0) / DLE)
    return np.clip(np.where(np.isfinite(b), b, 0), 0, NB - 1).astype(np.int64)


def features(rows, bounds):
    """rows [n][5] float32 trial log -> x [n][4] float32, y [n] float32, entry [n]."""
    r = np.asarray(rows, dtype=np.float32).astype(np.float64)
    lnt, lne, z, ent, lnw = r[:, 0], r[:, 1], r[:, 2], r[:, 3].astype(np.int64), r[:, 4]
    x = np.stack([(lnt - 10.0) / 10.0, (lne + 7.0) / 7.0, 2.0 * z - 1.0, (ent - 40.0) / 32.0], axis=1)
    y = lnw - np.log(np.asarray(bounds)[ent, eta_bin_of_ln(lne)])
    return x.astype(np.float32), y.astype(np.float32), ent


def forward(theta, x, dtype=np.float32, round_bf16=True):
    """Network output f [n].  round_bf16: weights and the first hidden layer in
    bfloat16 (the kernels' arithmetic); False: the plain function in `dtype`."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float32))
    if round_bf16:
        W1, b1, W2, b2, W3 = bf16(W1), bf16(b1), bf16(W2), bf16(b2), bf16(W3)
    x = np.asarray(x, dtype=dtype)
    a1 = x @ W1.T.astype(dtype) + b1.astype(dtype)
    h1 = np.maximum(a1, 0).astype(np.float32)
    if round_bf16:
        h1 = bf16(h1)
    a2 = h1.astype(dtype) @ W2.T.astype(dtype) + b2.astype(dtype)
    h2 = np.maximum(a2, 0)
    return (h2 @ W3.astype(dtype) + dtype(b3)).astype(dtype)


def loss_grad(theta, x, y, tau, round_bf16=True):
    """Pinball loss and its gradient with respect to the master parameters, FP64.

    With round_bf16 the function is the kernels' (bfloat16 weights and first
    hidden layer), differentiated with the roundings taken as the identity."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(a, dtype=np.float64) for a in unpack(np.asarray(theta, np.float32))]
    if round_bf16:
        W1, b1, W2, b2, W3 = [bf16(np.float32(a)).astype(np.float64) for a in (W1, b1, W2, b2, W3)]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    h1q = bf16(h1.astype(np.float32)).astype(np.float64) if round_bf16 else h1
    a2 = h1q @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    f = h2 @ W3 + b3
    r = y - f
    loss = np.mean(np.where(r >= 0, tau * r, (tau - 1.0) * r))
    gf = -np.where(r >= 0, tau, tau - 1.0) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = gf @ h2
    g[OFF_B3] = gf.sum()
    da2 = np.outer(gf, W3) * (a2 > 0)
    g[OFF_W2:OFF_B2] = (da2.T @ h1q).ravel()
    g[OFF_B2:OFF_W3] = da2.sum(axis=0)
    da1 = (da2 @ W2) * (a1 > 0)
    g[OFF_W1:OFF_B1] = (da1.T @ x).ravel()
    g[OFF_B1:OFF_W2] = da1.sum(axis=0)
    return loss, g


def grad_magnitudes(theta, x, y, tau, round_bf16=True):
    """Each gradient element's sum of the absolute values of its terms (the
    same sums as loss_grad with every factor replaced by its magnitude).  A
    sum of terms each rounded to relative error e is off by at most e times
    this: the scale against which a gradient computed with rounded
    (bfloat16) backward operands is compared element by element."""
    W1, b1, W2, b2, W3, b3 = [np.asarray(a, dtype=np.float64) for a in unpack(np.asarray(theta, np.float32))]
    if round_bf16:
        W1, b1, W2, b2, W3 = [bf16(np.float32(a)).astype(np.float64) for a in (W1, b1, W2, b2, W3)]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.shape[0]
    a1 = x @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    h1q = bf16(h1.astype(np.float32)).astype(np.float64) if round_bf16 else h1
    a2 = h1q @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    f = h2 @ W3 + b3
    r = y - f
    gf = np.abs(np.where(r >= 0, tau, tau - 1.0)) / n
    g = np.zeros(NPARAM)
    g[OFF_W3:OFF_B3] = gf @ h2
    g[OFF_B3] = gf.sum()
    da2 = np.outer(gf, np.abs(W3)) * (a2 > 0)
    g[OFF_W2:OFF_B2] = (da2.T @ h1q).ravel()
    g[OFF_B2:OFF_W3] = da2.sum(axis=0)
    da1 = (da2 @ np.abs(W2)) * (a1 > 0)
    g[OFF_W1:OFF_B1] = (da1.T @ np.abs(x)).ravel()
    g[OFF_B1:OFF_W2] = da1.sum(axis=0)
    return g


def adam_step(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), step counted from 1; FP64 reference."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def cell_ids(rows, cell_edges):
    """Cell of each logged trial: (entry - 8) * 384 + eta bin * 8 + ln t cell,
    the ln t cell the largest k in 1..7 with edge[k] < ln t, else 0 (the cell
    the shower takes for that scale)."""
    r = np.asarray(rows, dtype=np.float32).astype(np.float64)
    ent = np.clip(r[:, 3].astype(np.int64), IS0, IS0 + NENT_IS - 1) - IS0
    E = np.asarray(cell_edges, dtype=np.float64)
    k = np.zeros(len(r), dtype=np.int64)
    for j in range(1, NTB):
        k = np.where(E[j] < r[:, 0], j, k)
    return (ent * NB + eta_bin_of_ln(r[:, 1])) * NTB + k


def calibrate(theta, x, y, cell, round_bf16=True):
    """Margins delta[64][48][8] (+inf: the analytic bound) from held-out rows
    with their cells, and the row count of each cell."""
    f = forward(theta, x, round_bf16=round_bf16).astype(np.float64)
    res = np.asarray(y, dtype=np.float64) - f
    cell = np.asarray(cell, dtype=np.int64)
    ncell = NENT_IS * NB * NTB
    mx = np.full(ncell, -np.inf)
    np.maximum.at(mx, cell, res)
    cnt = np.bincount(cell, minlength=ncell)
    mx3, cnt3 = mx.reshape(NENT_IS, NB, NTB), cnt.reshape(NENT_IS, NB, NTB)
    mxb, cntb = mx3.max(axis=2), cnt3.sum(axis=2)
    mxe, cnte = mxb.max(axis=1), cntb.sum(axis=1)
    d_ent = np.where(cnte >= MIN_CAL, mxe + CAL_MARGIN, np.inf)
    d_bin = np.where(cntb >= MIN_CAL_BIN, mxb + CAL_MARGIN, d_ent[:, None])
    delta = np.where(cnt3 >= MIN_CAL_CELL, mx3 + CAL_MARGIN, d_bin[:, :, None])
    # an entry without enough rows keeps the analytic bound in every cell
    delta = np.where(np.isfinite(d_ent)[:, None, None], delta, np.inf)
    return delta, cnt3


def probe_features(cell_edges):
    """Probe inputs of every cell, [64*48*8*48][4] float32, cell-major."""
    E = np.asarray(cell_edges, dtype=np.float64)
    rows = np.zeros((NENT_IS, NB, NTB, NPT, NPE, NPZ, 4))
    for e in range(NENT_IS):
        for b in range(NB):
            lo = LNETA0 + b * DLE
            lne = (lo, lo + DLE)
            etalo = math.exp(lo)
            for k in range(NTB):
                lnt = (E[k], 0.5 * (E[k] + E[k + 1]), E[k + 1])
                for i, lt in enumerate(lnt):
                    for j, le in enumerate(lne):
                        for q in range(NPZ):
                            z = etalo + (1.0 - etalo) * (q / (NPZ - 1.0))
                            rows[e, b, k, i, j, q] = ((lt - 10.0) / 10.0, (le + 7.0) / 7.0,
                                                      2.0 * z - 1.0, (e + IS0 - 40.0) / 32.0)
    return rows.reshape(-1, 4).astype(np.float32)


def up6(v):
    """Round positive values up onto m * 2^e with m a multiple of 1/128 in [1/2, 1]."""
    m, e = np.frexp(np.asarray(v, dtype=np.float64))
    return np.ldexp(np.ceil(m * 128.0) / 128.0, e)


def tabulate(theta, delta, bounds, cell_edges, fmax=None):
    """The learned bound table [64][48][8] (doubles).  fmax: the per-cell maximum
    of the network over the probe points, computed here if not given."""
    if fmax is None:
        f = forward(theta, probe_features(cell_edges))
        fmax = f.reshape(NENT_IS, NB, NTB, NPROBE).max(axis=3)
    R = np.asarray(bounds, dtype=np.float64)[IS0:IS0 + NENT_IS, :, None]
    d = np.asarray(delta, dtype=np.float64)
    if d.ndim == 1:  # one margin per entry
        d = d[:, None, None]
    v = np.clip(d + fmax.astype(np.float64), V_MIN, 0.0)
    tab = np.where(np.isfinite(d), np.minimum(R, up6(R * np.exp(v))), R)
    return np.ascontiguousarray(np.broadcast_to(tab, (NENT_IS, NB, NTB)), dtype=np.float64)


def train(theta, x, y, steps, batch, lr, tau, seed=0, round_bf16=True):
    """Reference training loop (FP64 Adam over random batches); returns theta."""
    rng = np.random.Generator(np.random.Philox(seed))
    th = np.asarray(theta, dtype=np.float64).copy()
    m = np.zeros(NPARAM)
    v = np.zeros(NPARAM)
    for s in range(1, steps + 1):
        idx = rng.integers(0, x.shape[0], size=batch)
        _, g = loss_grad(th.astype(np.float32), x[idx], y[idx], tau, round_bf16)
        th, m, v = adam_step(th, m, v, g, s, lr)
    return th.astype(np.float32)

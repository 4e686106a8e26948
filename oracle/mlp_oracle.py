"""Plain FP64 oracle of the learned closure: features, MLP forward/backward, Adam, and the
closure-residual loss.  TEST INFRASTRUCTURE ONLY (tests, smoke, CPU baseline).

The paper replaces the closure by a fully-connected network evaluated as batched matrix
products with standardised inputs and outputs (Sec. "Phase 1-2", "Phase 3"; Adam, MSE,
StandardScaler).  Here the inputs are the theta-normalised central moments (Galilean and
scale invariant) and the targets the normalised coefficients:
  features  [P/th - I (6), T/th^1.5 (10), R/th^2 - 5 I (6), W/th^2.5 (3), eps_hat, log10 N]
  targets   [tau Ct - 5 eps_hat I (6), tau sqrt(th) Gamma (3)]
The network is 32 -> 128 -> 128 -> 128 -> 16 (27 features and 9 targets, zero padded),
SiLU activations, linear output.

Flat FP32 parameter vector (shared layout with the GPU library's network buffer):
  W1[128][32] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[16][128] b4[16]
  x_mean[32] x_std[32] y_mean[16] y_std[16]
"""
import numpy as np

NF, NH, NO = 32, 128, 16
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NO, NH)), ("b4", (NO,)),
          ("x_mean", (NF,)), ("x_std", (NF,)), ("y_mean", (NO,)), ("y_std", (NO,))]
N_TRAIN = NH * NF + NH + 2 * (NH * NH + NH) + NO * NH + NO   # trainable prefix: 39312
N_PARAMS = N_TRAIN + 2 * NF + 2 * NO                         # 39408

S2 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[n], dtype=np.float64).ravel() for n, _ in SHAPES])


def bf16(a):
    """Round to bfloat16 (nearest, ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(mom, eps_hat):
    """[n][32] features of moment records [n][32] (zero padded beyond 27)."""
    mom = np.asarray(mom, dtype=np.float64)
    th = mom[:, 4]
    f = np.zeros((mom.shape[0], NF))
    P = mom[:, 5:11] / th[:, None]
    f[:, 0:6] = P - np.array([1, 0, 0, 1, 0, 1])
    f[:, 6:16] = mom[:, 11:21] / th[:, None] ** 1.5
    f[:, 16:22] = mom[:, 21:27] / th[:, None] ** 2 - 5 * np.array([1, 0, 0, 1, 0, 1])
    f[:, 22:25] = mom[:, 27:30] / th[:, None] ** 2.5
    f[:, 25] = eps_hat
    f[:, 26] = np.log10(mom[:, 0])
    return f


def targets(rec, eps_hat):
    """[n][16] normalised targets of exact update records (zero padded beyond 9)."""
    rec = np.asarray(rec, dtype=np.float64)
    tau, th = rec[:, 9], rec[:, 10]
    y = np.zeros((rec.shape[0], NO))
    y[:, 0:6] = rec[:, 0:6] * tau[:, None] - 5 * eps_hat * np.array([1, 0, 0, 1, 0, 1])
    y[:, 6:9] = rec[:, 6:9] * (tau * np.sqrt(th))[:, None]
    return y


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(p, xs, emulate_bf16=False):
    """Standardised inputs xs [n][32] -> standardised outputs [n][16] and the cache.
    With emulate_bf16 the weights, the input and every hidden activation are rounded
    to bfloat16 where the GPU stores them in that format; sums stay exact (FP64)."""
    q = (lambda a: bf16(a)) if emulate_bf16 else (lambda a: a)
    h = q(xs)
    cache = [h]
    zs = []
    for l in (1, 2, 3):
        z = h @ q(p[f"W{l}"]).T + p[f"b{l}"]
        zs.append(z)
        h = q(silu(z))
        cache.append(h)
    y = h @ q(p["W4"]).T + p["b4"]
    return y, (cache, zs)


def backward(p, cache, dy, emulate_bf16=False):
    """Gradients of sum(dy * y) w.r.t. the trainable parameters (dict).  With
    emulate_bf16 the output gradients and pre-activation gradients enter the products in
    bfloat16, as on the GPU; bias gradients sum them unrounded."""
    q = (lambda a: bf16(a)) if emulate_bf16 else (lambda a: a)
    hs, zs = cache
    g = {}
    d = dy
    g["W4"] = q(d).T @ hs[3]
    g["b4"] = d.sum(0)
    dh = q(d) @ q(p["W4"])
    for l in (3, 2, 1):
        dz = dh * dsilu(zs[l - 1])
        g[f"W{l}"] = q(dz).T @ hs[l - 1]
        g[f"b{l}"] = dz.sum(0)
        if l > 1:
            dh = q(dz) @ q(p[f"W{l}"])
    return g


def mse_grad(y, t, mask):
    """Loss mean over samples of sum over the masked outputs of (y - t)^2, and dL/dy."""
    n = y.shape[0]
    d = (y - t) * mask[None, :]
    return float((d * d).sum() / n), 2.0 * d / n


def adam(p_flat, g_flat, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on the trainable prefix; returns new (p, m, v)."""
    p, m, v = p_flat.copy(), m.copy(), v.copy()
    g = g_flat[:N_TRAIN]
    m[:N_TRAIN] = b1 * m[:N_TRAIN] + (1 - b1) * g
    v[:N_TRAIN] = b2 * v[:N_TRAIN] + (1 - b2) * g * g
    mh = m[:N_TRAIN] / (1 - b1**t)
    vh = v[:N_TRAIN] / (1 - b2**t)
    p[:N_TRAIN] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def grads_flat(g):
    out = np.zeros(N_PARAMS)
    o = 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        if name in g:
            out[o:o + n] = g[name].ravel()
        o += n
    return out


# ---------------------------------------------------------------------------------------
# Coefficient-sensitivity probe (Sec. "Heuristic coefficient-sensitivity probe"): npass
# forward passes with an inference-time dropout mask of rate p on the hidden activations;
# per coefficient the standard deviation over the passes (1/N, about the mean of the
# passes), and per cell the Euclidean norms of the deviations of the stress block and of
# the heat-flux block.
#
# Readings: the perturbed outputs are the de-standardised normalised coefficients
# [tau Ct - 5 eps_hat I (6), tau sqrt(th) Gamma (3)]; dropout is inverted (kept
# activations scaled by 1/(1-p)) and acts after the SiLU of each of the three hidden
# layers, not on the input or the output; the masks come from Philox4x32-10 (Salmon et
# al., SC'11) keyed by the seed (low word, high word) with counter (cell, pass, 6,
# 32 (layer-1) + unit // 4), word unit % 4 deciding hidden unit `unit`; a unit is dropped
# when that word is below floor(p 2^32).  Cells without features (N <= 1 or theta <= 0)
# report zero.

PHILOX_M = (0xD2511F53, 0xCD9E8D57)
PHILOX_W = (0x9E3779B9, 0xBB67AE85)
PURPOSE_DROPOUT = 6


def philox(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on arrays of counters (uint64 arrays holding 32-bit words)."""
    m32 = np.uint64(0xFFFFFFFF)
    x = [np.asarray(v, dtype=np.uint64) & m32 for v in (c0, c1, c2, c3)]
    k = [np.uint64(int(k0) & 0xFFFFFFFF), np.uint64(int(k1) & 0xFFFFFFFF)]
    for r in range(10):
        if r:
            k = [(k[0] + np.uint64(PHILOX_W[0])) & m32, (k[1] + np.uint64(PHILOX_W[1])) & m32]
        p0 = np.uint64(PHILOX_M[0]) * x[0]
        p1 = np.uint64(PHILOX_M[1]) * x[2]
        x = [(p1 >> np.uint64(32)) ^ x[1] ^ k[0], p1 & m32, (p0 >> np.uint64(32)) ^ x[3] ^ k[1],
             p0 & m32]
    return x


def dropout_keep(seed, ncell, npass, p, cells=None):
    """keep[cell][pass][layer-1][unit] of the three hidden layers (bool); cells: the cell
    indices of the rows (default 0 .. ncell-1)."""
    ids = np.arange(ncell) if cells is None else np.asarray(cells)
    cell, pss, sub = np.meshgrid(ids, np.arange(npass), np.arange(3 * NH // 4), indexing="ij")
    w = philox(cell, pss, np.full_like(cell, PURPOSE_DROPOUT), sub, seed & 0xFFFFFFFF, seed >> 32)
    words = np.stack(w, axis=-1).reshape(ncell, npass, 3, NH)
    return words >= np.uint64(int(np.floor(p * 2.0**32)))


def dropout_sensitivity(p_flat, mom, eps_hat, npass, p, seed, emulate_bf16=True, cells=None):
    """sens[n][2] = (sigma_Stress, sigma_Heat) of moment records mom[n][32]; cells: the
    cell index of every record (default 0 .. n-1), which keys its dropout masks."""
    P = unpack(p_flat)
    mom = np.asarray(mom, dtype=np.float64)
    n = mom.shape[0]
    valid = (mom[:, 0] > 1.0) & (mom[:, 4] > 0.0)
    f = np.zeros((n, NF))
    if valid.any():
        f[valid] = features(mom[valid], eps_hat)
    xs = (f - P["x_mean"]) / P["x_std"]
    keep = dropout_keep(seed, n, npass, p, cells)
    scale = 1.0 / (1.0 - p)
    q = (lambda a: bf16(a)) if emulate_bf16 else (lambda a: a)
    ys = np.zeros((npass, n, 9))
    for k in range(npass):
        h = q(xs)
        for l in (1, 2, 3):
            a = silu(h @ q(P[f"W{l}"]).T + P[f"b{l}"])
            h = q(np.where(keep[:, k, l - 1, :], a * scale, 0.0))
        y = h @ q(P["W4"]).T + P["b4"]
        ys[k] = (y * P["y_std"] + P["y_mean"])[:, :9]
    sigma = ys.std(axis=0)
    sens = np.stack([np.sqrt((sigma[:, :6] ** 2).sum(1)), np.sqrt((sigma[:, 6:] ** 2).sum(1))], 1)
    sens[~valid] = 0.0
    return sens

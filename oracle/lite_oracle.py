"""Plain FP64 oracle of the paper's LITE surrogate: its 16 low-order inputs, its targets,
and the 16-256-256-256-256-9 ReLU network (forward, backward, the MSE of standardised
targets, Adam).  TEST INFRASTRUCTURE ONLY (tests, smoke, CPU baseline).

Sec. "Phase 1-2": the inputs are rho, T, U_x, U_y, U_z, Pi_xx, Pi_xy, Pi_xz, Pi_yy, Pi_yz,
Pi_zz, q_x, q_y, q_z, DM2, nu and the targets the six C_ij and the three Gamma_i; Sec.
"Neural Network Architecture": four ReLU hidden layers of 256 units between the 16 inputs
and a linear 9-output regression head (204,041 trainable parameters); inputs and outputs
are standardised by per-column mean and standard deviation (Sec. "Phase 3").

Readings of what the paper leaves undefined (stated once here, used everywhere):
  * rho = n m with n = N fnum / V_cell (the cell's real number density), T = theta m / k_B;
  * Pi_ij = rho (P_ij - theta delta_ij), the deviatoric stress of the cell's particles;
  * q_i = rho <c_i |c|^2> / 2, the heat flux;
  * DM2 = <|c|^2> = 3 theta, the second central moment (DM6 of the cavity diagnostics is
    <|c|^6>, and the stability table lists DM2 among quantities that must stay positive);
  * nu = 1 / tau = p / (2 mu(T)), the collision frequency of eq. tau;
  * targets: Ct_ij (= c^(1)_ij + delta_ij / tau, the coefficient eq. update_N applies) and
    Gamma_i, in solver units; Ct differs from c^(1) by delta_ij nu, which the inputs fix,
    and leaves out the large -1/tau that would swamp the learned part in BF16.

Flat FP32 parameter vector (the layout of the GPU library's LITE network buffer):
  W1[256][16] b1[256] W2[256][256] b2[256] W3[256][256] b3[256] W4[256][256] b4[256]
  W5[16][256] b5[16] x_mean[16] x_std[16] y_mean[16] y_std[16]
The output layer is padded from 9 to 16 rows (rows 9..15 zero); the trainable prefix is
everything before x_mean.
"""
import numpy as np

NF, NH, NLAYER, NO = 16, 256, 5, 16
SHAPES = [("W1", (NH, NF)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NH)), ("b3", (NH,)), ("W4", (NH, NH)), ("b4", (NH,)),
          ("W5", (NO, NH)), ("b5", (NO,)),
          ("x_mean", (NF,)), ("x_std", (NF,)), ("y_mean", (NO,)), ("y_std", (NO,))]
N_TRAIN = NH * NF + NH + 3 * (NH * NH + NH) + NO * NH + NO      # 205840
N_PARAMS = N_TRAIN + 2 * NF + 2 * NO                            # 205904
PAPER_PARAMS = NH * NF + NH + 3 * (NH * NH + NH) + 9 * NH + 9   # 204041 (unpadded head)

S2 = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
DELTA6 = np.array([1.0, 0.0, 0.0, 1.0, 0.0, 1.0])


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
    """Round to bfloat16 (nearest, ties to even) through FP32, returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def tau_of(w, n_dens, theta):
    """tau = 2 mu / p (eq. tau) with the VHS viscosity mu = mu_ref (T / T_ref)^omega."""
    T = theta * w["mass"] / w["kB"]
    p = n_dens * w["kB"] * T
    mu = w["mu_ref"] * (T / w["T_ref"]) ** w["omega"]
    return 2.0 * mu / p


def features(w, mom, nvol=None):
    """[n][16] inputs of moment records mom[n][32] (layout of the library's records):
    rho, T, U (3), Pi (11 12 13 22 23 33), q (3), DM2, nu.  nvol: real molecules per
    particle over the cell volume, per record (default the workload's fnum_over_vol)."""
    mom = np.asarray(mom, dtype=np.float64)
    n = mom.shape[0]
    N, th = mom[:, 0], mom[:, 4]
    nv = np.full(n, float(w["fnum_over_vol"])) if nvol is None else np.asarray(nvol, dtype=np.float64)
    ndens = N * nv
    rho = ndens * w["mass"]
    f = np.zeros((n, NF))
    f[:, 0] = rho
    f[:, 1] = th * w["mass"] / w["kB"]
    f[:, 2:5] = mom[:, 1:4]
    f[:, 5:11] = rho[:, None] * (mom[:, 5:11] - th[:, None] * DELTA6)
    T = mom[:, 11:21]     # T111 T112 T113 T122 T123 T133 T222 T223 T233 T333
    S = np.stack([T[:, 0] + T[:, 3] + T[:, 5], T[:, 1] + T[:, 6] + T[:, 8],
                  T[:, 2] + T[:, 7] + T[:, 9]], 1)
    f[:, 11:14] = 0.5 * rho[:, None] * S
    f[:, 14] = 3.0 * th
    f[:, 15] = 1.0 / tau_of(w, ndens, th)
    return f


def targets(rec):
    """[n][16] targets (Ct_ij (6), Gamma_i (3), zero padded) of update records."""
    rec = np.asarray(rec, dtype=np.float64)
    y = np.zeros((rec.shape[0], NO))
    y[:, 0:9] = rec[:, 0:9]
    return y


def relu(z):
    return np.maximum(z, 0.0)


def forward(p, xs, emulate_bf16=False):
    """Standardised inputs xs [n][16] -> standardised outputs [n][16] and the cache.
    With emulate_bf16 the weights, the input and every hidden activation are rounded to
    bfloat16 where the GPU holds them in that format; the sums are exact (FP64)."""
    q = bf16 if emulate_bf16 else (lambda a: a)
    h = q(xs)
    hs, zs = [h], []
    for layer in range(1, NLAYER):
        z = h @ q(p[f"W{layer}"]).T + p[f"b{layer}"]
        zs.append(z)
        h = q(relu(z))
        hs.append(h)
    y = h @ q(p[f"W{NLAYER}"]).T + p[f"b{NLAYER}"]
    return y, (hs, zs)


def backward(p, cache, dy, emulate_bf16=False):
    """Gradients of sum(dy * y) w.r.t. the trainable parameters (dict).  With
    emulate_bf16 the output and pre-activation gradients enter the products in bfloat16
    as on the GPU; the bias gradients sum them unrounded.  ReLU'(0) = 0."""
    q = bf16 if emulate_bf16 else (lambda a: a)
    hs, zs = cache
    g = {}
    d = dy
    L = NLAYER
    g[f"W{L}"] = q(d).T @ hs[L - 1]
    g[f"b{L}"] = d.sum(0)
    dh = q(d) @ q(p[f"W{L}"])
    for layer in range(L - 1, 0, -1):
        dz = dh * (zs[layer - 1] > 0.0)
        g[f"W{layer}"] = q(dz).T @ hs[layer - 1]
        g[f"b{layer}"] = dz.sum(0)
        if layer > 1:
            dh = q(dz) @ q(p[f"W{layer}"])
    return g


def mse_grad(y, t, mask):
    """Mean over samples of the masked squared error, and its gradient w.r.t. y."""
    n = y.shape[0]
    d = (y - t) * mask[None, :]
    return float((d * d).sum() / n), 2.0 * d / n


def grads_flat(g):
    out = np.zeros(N_PARAMS)
    o = 0
    for name, shp in SHAPES:
        n = int(np.prod(shp))
        if name in g:
            out[o:o + n] = g[name].ravel()
        o += n
    return out


def adam(p_flat, g_flat, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma and Ba) on the trainable prefix; returns new (p, m, v)."""
    p, m, v = p_flat.copy(), m.copy(), v.copy()
    g = g_flat[:N_TRAIN]
    m[:N_TRAIN] = b1 * m[:N_TRAIN] + (1 - b1) * g
    v[:N_TRAIN] = b2 * v[:N_TRAIN] + (1 - b2) * g * g
    mh = m[:N_TRAIN] / (1 - b1 ** t)
    vh = v[:N_TRAIN] / (1 - b2 ** t)
    p[:N_TRAIN] -= lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def standardise(f, P, emulate_fp32=False):
    """(f - x_mean) / x_std; with emulate_fp32 the inputs are first stored as FP32 and the
    standardisation is done in FP32, as the GPU forms its network input."""
    if not emulate_fp32:
        return (f - P["x_mean"]) / P["x_std"]
    f32 = np.asarray(f).astype(np.float32)
    return ((f32 - P["x_mean"].astype(np.float32)) / P["x_std"].astype(np.float32)).astype(np.float64)


def coefficients(w, p_flat, mom, nvol=None, emulate_bf16=True):
    """The LITE closure of moment records: (Ct [n][6], Gamma [n][3], valid [n]) from the
    de-standardised network outputs; cells without features (N <= 1 or theta <= 0) are
    not valid.  With emulate_bf16 the network input is also formed in FP32 (standardise)."""
    P = unpack(p_flat)
    mom = np.asarray(mom, dtype=np.float64)
    valid = (mom[:, 0] > 1.0) & (mom[:, 4] > 0.0)
    f = np.zeros((mom.shape[0], NF))
    if valid.any():
        f[valid] = features(w, mom[valid], None if nvol is None else np.asarray(nvol)[valid])
    y, _ = forward(P, standardise(f, P, emulate_bf16), emulate_bf16)
    d = y * P["y_std"] + P["y_mean"]
    return d[:, 0:6], d[:, 6:9], valid

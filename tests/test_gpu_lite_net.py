"""The paper's LITE surrogate on the GPU (16 low-order inputs, 16-256x4-9 ReLU network,
BF16 MFMA with FP32 accumulation) against the FP64 oracle of oracle/lite_oracle.py, which
rounds to bfloat16 where the GPU holds bfloat16 values (weights, inputs, hidden
activations, back-propagated gradients in the products).  The remaining differences are
FP32 against FP64 accumulation and the bfloat16 rounding flips they cause now and then
(one bfloat16 ulp of one activation, carried through the later layers); the oracle forms
the network input as the kernel does (inputs stored as FP32, standardised in FP32).  Every
bound below is element by element and its measured maximum is printed; on an MI355X:
outputs within 8.1e-3 of their rms everywhere (0.43 of the bound) and within 1e-3 in
99.5 % of the cells (the rest carry a flip through the later layers), closure records within
7.3e-3, gradients within 3.5e-4 of their tensor's rms."""
import numpy as np
import pytest
import torch

from oracle import lite_oracle as L
from oracle import oracle as O
from paper_2606_15622_amd import inputs as I

pytestmark = pytest.mark.gpu


def fp():
    from paper_2606_15622_amd import fpgpu
    fpgpu.load()
    return fpgpu


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def cells(ncell, seed):
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, 400, ncell)
    counts[:7] = [0, 1, 2, 3, 4, 5, 6]
    vx, vy, vz, off = I.mixture_cells(counts, seed=seed)
    return O.moments(off, vx, vy, vz)


def params_for(w, mom, seed):
    """He-initialised weights, scalers fitted to the oracle's inputs and targets of mom."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shp in L.SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shp) * np.sqrt(2.0 / shp[1])
        elif name.startswith("b"):
            d[name] = rng.standard_normal(shp) * 0.05
    d["W5"][9:] = 0.0
    d["b5"][9:] = 0.0
    ok = (mom[:, 0] > 1) & (mom[:, 4] > 0)
    f = L.features(w, mom[ok])
    d["x_mean"] = f.mean(0)
    d["x_std"] = np.where(f.std(0) > 0, f.std(0), 1.0)
    d["y_mean"] = np.zeros(16)
    d["y_std"] = np.ones(16)
    d["y_mean"][:9] = rng.standard_normal(9) * 1e5
    d["y_std"][:9] = rng.uniform(1e5, 1e6, 9)
    return L.pack(d).astype(np.float32)


def bound_stats(yg, yo, rel, floor):
    err = np.abs(yg - yo)
    rms = np.sqrt((yo ** 2).mean(0))
    lim = rel * np.abs(yo) + floor * rms
    return err, rms, lim


def test_inputs_and_targets_match_oracle():
    F = fp()
    nc = 3001
    w = I.cavity(kn=0.5, ncell=1)
    mom = cells(nc, 2)
    ok = (mom[:, 0] > 1) & (mom[:, 4] > 0)
    ctx = F.Context(w, 1)
    md = dev(mom[ok], torch.float64)
    n = int(ok.sum())
    feats = torch.zeros((n, 16), dtype=torch.float32, device="cuda")
    ctx.lite_features(md, n, feats)
    wex = I.couette(ncell=nc, eps_hat=0.01)
    rec, st = O.closure(wex, mom)
    tg = torch.zeros((nc, 16), dtype=torch.float32, device="cuda")
    ctx.lite_targets(dev(rec, torch.float64), nc, tg)
    torch.cuda.synchronize()
    fo = L.features(w, mom[ok])
    fg = feats.double().cpu().numpy()
    scale = np.abs(fo).max(0)
    # FP64 arithmetic on both sides, then one rounding to FP32 on the GPU
    assert np.all(np.abs(fg - fo) <= 2.0 ** -23 * np.abs(fo) + 1e-12 * scale)
    np.testing.assert_array_equal(tg.cpu().numpy(), L.targets(rec).astype(np.float32))


def test_inference_matches_bf16_oracle():
    F = fp()
    nc = 2000 + 37
    w = I.cavity(kn=0.5, ncell=1)
    w = dict(w, geometry="couette1d", nx=nc, ny=1, lx=w["dx"] * nc, ly=1.0, dy=1.0)
    mom = cells(nc, 3)
    pflat = params_for(w, mom, 1)
    ctx = F.Context(w, 1)
    net = F.LiteNetwork(ctx, 0)
    net.load(dev(pflat, torch.float32))
    y = torch.full((nc, 16), 7.0, dtype=torch.float32, device="cuda")
    net.infer(dev(mom, torch.float64), y)
    torch.cuda.synchronize()
    yg = y.double().cpu().numpy()
    P = L.unpack(pflat.astype(np.float64))
    ok = (mom[:, 0] > 1) & (mom[:, 4] > 0)
    f = np.zeros((nc, 16))
    f[ok] = L.features(w, mom[ok])
    yo, _ = L.forward(P, L.standardise(f, P, emulate_fp32=True), emulate_bf16=True)
    assert np.all(yg[:, 9:] == 0)
    err, rms, lim = bound_stats(yg[:, :9], yo[:, :9], 2.0 ** -7, 2.0 ** -6)
    tight = np.all(err <= 1e-3 * (np.abs(yo[:, :9]) + rms), 1).mean()
    print(f"\nLITE inference: max err / rms {float((err / rms).max()):.3e}, "
          f"max err / bound {float((err / lim).max()):.3e}, cells within 1e-3: {tight:.4f}")
    assert np.all(err <= lim)
    assert tight >= 0.99


def test_closure_records_and_forced_fallback():
    F = fp()
    nc = 1500 + 11
    w = I.couette(ncell=nc, eps_hat=0.01)
    mom = cells(nc, 4)
    pflat = params_for(w, mom, 2)
    ctx = F.Context(w, 1)
    net = F.LiteNetwork(ctx, 0)
    net.load(dev(pflat, torch.float32))
    md = dev(mom, torch.float64)
    rec = torch.zeros((nc, 16), dtype=torch.float64, device="cuda")
    st = torch.zeros(nc, dtype=torch.int32, device="cuda")
    net.closure(md, rec, st, float("inf"), 0.0)
    rex = torch.zeros_like(rec)
    sex = torch.zeros_like(st)
    ctx.closure_solve(md, rex, sex)
    r2 = torch.zeros_like(rec)
    s2 = torch.zeros_like(st)
    net.closure(md, r2, s2, 0.0, 0.0)
    torch.cuda.synchronize()
    g, stg = rec.cpu().numpy(), st.cpu().numpy()
    orec, ost = O.closure(w, mom)
    # statuses: the network's for solvable cells, the exact closure's otherwise
    solv = ost == O.OR_OK
    assert np.all(stg[solv] == F.CELL_NN) and np.all(stg[~solv] == ost[~solv])
    np.testing.assert_allclose(g[:, 9:14], orec[:, 9:14], rtol=1e-12, atol=1e-300)
    # the record's coefficients, re-standardised, against the oracle's outputs
    Ct, Gm, valid = L.coefficients(w, pflat.astype(np.float64), mom)
    P = L.unpack(pflat.astype(np.float64))
    yo = (np.concatenate([Ct, Gm], 1) - P["y_mean"][:9]) / P["y_std"][:9]
    yg = (g[:, :9] - P["y_mean"][:9]) / P["y_std"][:9]
    err, rms, lim = bound_stats(yg[solv], yo[solv], 2.0 ** -7, 2.0 ** -6)
    print(f"\nLITE closure records: max err / rms {float((err / rms).max()):.3e}")
    assert np.all(err <= lim)
    # tol 0: every solvable cell falls back to the exact solve, bit for bit
    sb = s2.cpu().numpy()
    assert np.all(sb[solv] == F.CELL_NN_FALLBACK)
    np.testing.assert_array_equal(r2.cpu().numpy()[:, :14], rex.cpu().numpy()[:, :14])


def test_gradient_matches_bf16_oracle():
    F = fp()
    B = 2048 + 5
    rng = np.random.default_rng(9)
    d = {}
    for name, shp in L.SHAPES:
        if name.startswith("W"):
            d[name] = rng.standard_normal(shp) * np.sqrt(2.0 / shp[1])
        elif name.startswith("b"):
            d[name] = rng.standard_normal(shp) * 0.05
        elif name.endswith("mean"):
            d[name] = rng.standard_normal(shp) * 0.3
        else:
            d[name] = rng.uniform(0.5, 2.0, shp)
    d["W5"][9:] = 0.0
    d["b5"][9:] = 0.0
    pflat = L.pack(d).astype(np.float32)
    feats = rng.standard_normal((B, 16)).astype(np.float32) * 2.0
    tg = np.zeros((B, 16), dtype=np.float32)
    tg[:, :9] = rng.standard_normal((B, 9)).astype(np.float32)
    w = I.couette(ncell=1)
    ctx = F.Context(w, 1)
    net = F.LiteNetwork(ctx, B)
    pd = dev(pflat, torch.float32)
    fd, td = dev(feats, torch.float32), dev(tg, torch.float32)
    grad = torch.zeros(F.LITE_PARAMS, dtype=torch.float32, device="cuda")
    grad2 = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.grad(pd, fd, td, B, grad, loss)
    net.grad(pd, fd, td, B, grad2, loss)
    torch.cuda.synchronize()
    assert torch.equal(grad, grad2)
    g = grad.double().cpu().numpy()
    P = L.unpack(pflat.astype(np.float64))
    y, cache = L.forward(P, L.standardise(feats.astype(np.float64), P, emulate_fp32=True),
                         emulate_bf16=True)
    ts = (tg.astype(np.float64) - P["y_mean"]) / P["y_std"]
    lo, dy = L.mse_grad(y, ts, np.r_[np.ones(9), np.zeros(7)])
    go = L.grads_flat(L.backward(P, cache, dy, emulate_bf16=True))
    assert float(loss.cpu()) == pytest.approx(lo, rel=1e-3)
    o = 0
    worst = 0.0
    for name, shp in L.SHAPES[:10]:
        n = int(np.prod(shp))
        ge, gr = g[o:o + n], go[o:o + n]
        rms = float(np.sqrt((gr ** 2).mean()))
        e = np.abs(ge - gr) / rms
        worst = max(worst, float(e.max()))
        assert np.all(e <= 2.0 ** -6), (name, float(e.max()))
        o += n
    print(f"\nLITE gradient: max |err| / tensor rms {worst:.3e}")
    assert np.all(g[L.N_TRAIN:] == 0)


def test_adam_matches_oracle():
    F = fp()
    ctx = F.Context(I.couette(ncell=1), 1)
    rng = np.random.default_rng(11)
    p = rng.standard_normal(L.N_PARAMS).astype(np.float32)
    m = np.zeros(L.N_PARAMS, dtype=np.float32)
    v = np.zeros(L.N_PARAMS, dtype=np.float32)
    pd, md, vd = dev(p, torch.float32), dev(m, torch.float32), dev(v, torch.float32)
    po, mo, vo = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in range(1, 4):
        g = rng.standard_normal(L.N_PARAMS).astype(np.float32)
        ctx.lite_adam(pd, dev(g, torch.float32), md, vd, t, 1e-3)
        po, mo, vo = L.adam(po, g.astype(np.float64), mo, vo, t, 1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(pd.cpu().numpy(), po, rtol=1e-5, atol=1e-6)
    assert np.all(pd.cpu().numpy()[L.N_TRAIN:] == p[L.N_TRAIN:])

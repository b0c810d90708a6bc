"""GPU parity of the learned surrogate's kernels, through the C ABI, against
the FP64 reference in oracle.mlp:

* input rows bit-exact (neighbour choice and order, every bfloat16 feature)
  on a small tank, a dense random cloud and a slab with ghosts, with row
  subsets and out-of-range rows; the rows' FP32 pair-sum rates against the
  oracle's FP64 sums, and the flag for rows with more than 64 neighbours;
* forward pass, loss and every weight / bias gradient of the bfloat16 MFMA
  kernels against the FP64 MLP evaluated on the same bfloat16 tensors
  (normwise <= 5e-3; the kernels differ from it only by FP32 accumulation
  and the rare bfloat16 rounding of a value that sits on a rounding boundary),
  for batch sizes with ragged tiles and with split-K weight gradients;
* Adam against its definition, bfloat16 weight copies bit-exact;
* training targets bit-exact, the application of a prediction to FP32 ulps,
  the judge's sums against numpy;
* the fused advance against the unfused chain (features, GEMMs, apply), and
  at the 1.47M-particle workload against the oracle chain on sampled
  particles.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp as om
from paper_1210_1017_amd import cases, sph
from parity_util import announce, relnorm, ulp32

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

GRAD_TOL = 5e-3
def _scales(p, inv_dt=0.0):
    """(inv_len, inv_vel, rho_ref, inv_rho, r2f, inv_acc, inv_drho, inv_dt)"""
    return (np.float32(1.0 / p["h"]), np.float32(2.0), np.float32(1000.0), np.float32(0.1),
            np.float32((1.85 * p["h"]) ** 2), np.float32(0.1), np.float32(1e-3),
            np.float32(inv_dt))


def _with_prev(case, seed):
    """The case with previous-step values that differ from the current ones
    (seeded), so that the own block's previous-step differences are live."""
    rng = np.random.default_rng(seed)
    st = {k: v.copy() for k, v in case.state.items()}
    for k in ("vx", "vy", "vz"):
        st[k + "p"] = (st[k] + rng.uniform(-2e-3, 2e-3, size=st[k].shape)).astype(np.float32)
    st["rhop"] = (st["rho"] + rng.uniform(-0.3, 0.3, size=st["rho"].shape)).astype(np.float32)
    return cases.Case(case.name + "+prev", dict(case.params), st, case.pos64)


def _bf16_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).cuda()


def _f32(a):
    return a.float().cpu().numpy().astype(np.float64)


def _sorted_gpu(case):
    n = case.n
    ctx = sph.Context(case.params, n)
    cur = sph.DeviceState.from_numpy(case.state)
    out = sph.DeviceState.empty(n)
    ctx.sort(cur, out, n)
    return ctx, cur, out


def _compare_rows(got, want, name):
    """Every slot feature and the own block's plain values bit-exact; the four
    pair-sum features (FP32 sums on the GPU, FP64 in the oracle, both rounded
    to bfloat16) within one bfloat16 step."""
    plain = np.ones(sph.NN_IN, dtype=bool)
    plain[om.SUM_COLS] = False
    bad = np.nonzero(np.any(got[:, plain] != want[:, plain], axis=1))[0]
    assert bad.size == 0, (name, bad[:5])
    g, w = got[:, om.SUM_COLS], want[:, om.SUM_COLS]
    assert np.all(np.abs(g - w) <= 2.0 ** -7 * np.abs(w) + 1e-3), (name, np.abs(g - w).max())
    assert np.mean(g != w) < 0.02, name


FEATURE_CASES = {
    "small_tank": lambda: cases.perturb(cases.small_tank(), 3),
    "dense_cloud": lambda: cases.random_cloud(1500, 0.02, (0.22, 0.22, 0.22), seed=5),
    "small_slab": lambda: cases.perturb(cases.small_slab(), 4),
    "tank_prev": lambda: _with_prev(cases.perturb(cases.small_tank(), 3), 11),
}


@pytest.mark.parametrize("name", list(FEATURE_CASES))
def test_features_bit_exact(name):
    case = FEATURE_CASES[name]()
    p, n = case.params, case.n
    announce(f"nn features {name} n={n}")
    ctx, _, out = _sorted_gpu(case)
    n0 = ctx.counts()["n_label"][0]
    sc = _scales(p, 1.0 / 6e-5 if name.endswith("prev") else 0.0)
    X = torch.empty(max(n0, 1), sph.NN_IN, dtype=torch.bfloat16, device="cuda")
    R = torch.empty(max(n0, 1), 4, dtype=torch.float32, device="cuda")
    ctx.nn_features(out, None, n0, sc, X, rates=R)
    torch.cuda.synchronize()
    srt = oracle.sort_state(p, case.state)
    _, cnt = oracle.nn_rows(p, srt, np.arange(n0), sc[4], om.SLOTS)
    assert bool(ctx.status() & sph.STATUS_NN_LIST) == bool((cnt > om.SLOTS).any())
    want = om.features(p, srt, np.arange(n0), sc)
    got = _f32(X[:n0])
    _compare_rows(got, want, name)
    if name.endswith("prev"):   # the previous-step block is live
        assert np.abs(want[:, 522:526]).max() > 0.1
    # FP32 sums of a few dozen terms against FP64, normwise within the
    # single-step bound, relative to the pressure part (ap = rate - g for
    # fluid) and to the continuity rate
    rref = om.rates(p, srt, np.arange(n0), sc)
    rg = R[:n0].cpu().numpy().astype(np.float64)
    fl = srt["state"]["type"][:n0] == cases.FLUID
    ap = rref[:, :3] - np.where(fl[:, None], np.asarray(p["g"]), 0.0)
    assert np.linalg.norm(rg[:, :3] - rref[:, :3]) <= 1e-4 * np.linalg.norm(ap)
    assert relnorm(rg[:, 3], rref[:, 3]) <= 1e-4
    assert np.all(rg[~fl, :3] == 0.0)
    # a row subset with repeats and rows outside the label-0 prefix
    rng = np.random.default_rng(1)
    rows = rng.integers(0, n0, 300).astype(np.int32)
    rows[::37] = n0 + 3
    rows[5] = -1
    rt = torch.from_numpy(rows).cuda()
    Xs = torch.empty(len(rows), sph.NN_IN, dtype=torch.bfloat16, device="cuda")
    ctx.nn_features(out, rt, len(rows), sc, Xs)
    gs = _f32(Xs)
    inside = (rows >= 0) & (rows < n0)
    _compare_rows(gs[inside], want[rows[inside]], name + " subset")
    assert not gs[~inside].any()
    Rs = torch.empty(len(rows), 4, dtype=torch.float32, device="cuda")
    ctx.nn_features(out, rt, len(rows), sc, Xs, rates=Rs)
    rs = Rs.cpu().numpy()
    assert np.array_equal(rs[inside], R[:n0].cpu().numpy()[rows[inside]])
    assert not rs[~inside].any()


def _random_net(width, cap, seed, out_gain=1.0):
    net = sph.Mlp(width, cap, train=True)
    net.init(seed)
    rng = np.random.default_rng(seed + 1)
    arr = net.arrays()
    for l in range(sph.NN_LAYERS):
        arr[f"b{l}"] = (0.1 * rng.standard_normal(arr[f"b{l}"].shape)).astype(np.float32)
    arr["w3"] = (arr["w3"] * out_gain).astype(np.float32)
    net.load(arr)
    return net, arr


def _oracle_net(arr):
    W = [om.bf16_round(arr[f"w{l}"].astype(np.float64)) for l in range(sph.NN_LAYERS)]
    b = [arr[f"b{l}"].astype(np.float64) for l in range(sph.NN_LAYERS)]
    return W, b


@pytest.mark.parametrize("rows", [1, 63, 65, 1000, 5000])
def test_forward_backward_vs_oracle(rows):
    announce(f"mlp forward/backward rows={rows}")
    case = cases.small_tank()
    ctx = sph.Context(case.params, case.n)
    net, arr = _random_net(128, max(rows, 64), 7, out_gain=50.0)
    ctx.mlp_sync(net)
    rng = np.random.default_rng(rows)
    X64 = om.bf16_round(rng.standard_normal((rows, sph.NN_IN)))
    T64 = rng.standard_normal((rows, sph.NN_OUT)).astype(np.float32).astype(np.float64)
    wcol = (1.0, 0.5, 2.0, 1.5)
    X, T = _bf16_dev(X64), torch.from_numpy(T64.astype(np.float32)).cuda()
    Y = torch.empty(rows, sph.NN_OUT, device="cuda")
    ctx.mlp_forward(net, X, rows, Y)
    ctx.mlp_backward(net, X, rows, T, wcol)
    torch.cuda.synchronize()
    W, b = _oracle_net(arr)
    # the bfloat16 weight copies are the rounded masters
    for l in range(sph.NN_LAYERS):
        assert np.array_equal(_f32(net.wb[l]), W[l])
    Yo, cache = om.forward(W, b, X64, emulate=True)
    Lo, dYo = om.mse(Yo, T64, wcol)
    gWo, gbo = om.backward(W, cache, dYo, emulate=True)
    errs = {"y": relnorm(Y.cpu().numpy(), Yo),
            "loss": abs(float(net.loss.item()) - Lo) / Lo}
    for l in range(sph.NN_LAYERS):
        errs[f"gw{l}"] = relnorm(net.gw[l].cpu().numpy(), gWo[l])
        errs[f"gb{l}"] = relnorm(net.gb[l].cpu().numpy(), gbo[l])
    print(rows, errs, flush=True)
    for k, v in errs.items():
        assert v <= GRAD_TOL, (k, v)
    # and against the FP64 MLP without any intermediate rounding (looser:
    # the bfloat16 storage of activations and gradients is part of the method)
    Yp, cp = om.forward(W, b, X64)
    assert relnorm(Y.cpu().numpy(), Yp) <= 0.05


def test_adam_vs_definition():
    announce("mlp adam")
    case = cases.small_tank()
    ctx = sph.Context(case.params, case.n)
    rows = 777
    net, arr = _random_net(128, rows, 11, out_gain=20.0)
    ctx.mlp_sync(net)
    rng = np.random.default_rng(2)
    X = _bf16_dev(om.bf16_round(rng.standard_normal((rows, sph.NN_IN))))
    T = torch.from_numpy(rng.standard_normal((rows, 4)).astype(np.float32)).cuda()
    Y = torch.empty(rows, 4, device="cuda")
    w = [arr[f"w{l}"].astype(np.float64) for l in range(4)]
    bb = [arr[f"b{l}"].astype(np.float64) for l in range(4)]
    m = [np.zeros_like(x) for x in w]
    v = [np.zeros_like(x) for x in w]
    mb = [np.zeros_like(x) for x in bb]
    vb = [np.zeros_like(x) for x in bb]
    for t in (1, 2, 3):
        ctx.mlp_forward(net, X, rows, Y)
        ctx.mlp_backward(net, X, rows, T, (1, 1, 1, 1))
        gw = [net.gw[l].cpu().numpy().astype(np.float64) for l in range(4)]
        gb = [net.gb[l].cpu().numpy().astype(np.float64) for l in range(4)]
        ctx.mlp_adam(net, 1e-3, 0.9, 0.999, 1e-8, t)
        torch.cuda.synchronize()
        for l in range(4):
            w[l], m[l], v[l] = om.adam(w[l], m[l], v[l], gw[l], t, 1e-3)
            bb[l], mb[l], vb[l] = om.adam(bb[l], mb[l], vb[l], gb[l], t, 1e-3)
            gwl = net.w[l].cpu().numpy()
            assert np.max(np.abs(gwl - w[l])) <= 1e-6 * max(1.0, np.abs(w[l]).max()), (t, l)
            assert np.max(np.abs(net.b[l].cpu().numpy() - bb[l])) <= 1e-6, (t, l)
            assert np.array_equal(_f32(net.wb[l]), om.bf16_round(gwl.astype(np.float64)))
            # keep the reference on the GPU's masters so rounding does not accumulate
            w[l] = gwl.astype(np.float64)
            bb[l] = net.b[l].cpu().numpy().astype(np.float64)


def _by_id(st: dict) -> dict:
    out = {}
    for k, a in st.items():
        o = np.empty_like(a)
        o[st["id"]] = a
        out[k] = o
    return out


def test_targets_bit_exact():
    case = cases.perturb(cases.small_tank(), 5)
    n = case.n
    announce(f"nn targets n={n}")
    ctx, cur, A = _sorted_gpu(case)
    B = sph.DeviceState.empty(n)
    ctx.step(A, B, n, 0)
    where = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.nn_index(B.t["id"], n, where)
    rows = np.random.default_rng(3).integers(0, n, 500).astype(np.int32)
    T = torch.empty(500, 4, device="cuda")
    inv_dv, inv_dr = np.float32(123.25), np.float32(0.75)
    ctx.nn_targets(A, B, where, torch.from_numpy(rows).cuda(), 500, inv_dv, inv_dr, T)
    torch.cuda.synchronize()
    a, b = A.to_numpy(n), B.to_numpy(n)
    assert np.array_equal(where.cpu().numpy()[b["id"]], np.arange(n))
    want = om.targets(a, _by_id(b), rows, inv_dv, inv_dr)
    assert np.array_equal(T.cpu().numpy(), want)
    # with rates (seeded FP32 inputs) subtracted over a span
    rts = (np.random.default_rng(7).standard_normal((500, 4)) * [5, 5, 5, 300]).astype(np.float32)
    span = np.float32(2.37e-4)
    ctx.nn_targets(A, B, where, torch.from_numpy(rows).cuda(), 500, inv_dv, inv_dr, T,
                   rates=torch.from_numpy(rts).cuda(), span=float(span))
    torch.cuda.synchronize()
    want = om.targets(a, _by_id(b), rows, inv_dv, inv_dr, rts=rts, span=span)
    assert np.array_equal(T.cpu().numpy(), want)


def test_apply_and_status():
    case = cases.perturb(cases.small_slab(), 6)
    n = case.n
    announce(f"nn apply n={n}")
    ctx, cur, S = _sorted_gpu(case)
    n0 = ctx.counts()["n_label"][0]
    before = S.to_numpy(n)
    rng = np.random.default_rng(4)
    Y = rng.standard_normal((n0, 4)).astype(np.float32)
    dv, dr, dt4 = np.float32(0.01), np.float32(0.5), np.float32(4e-4)
    ctx.nn_apply(S, torch.from_numpy(Y).cuda(), n0, dv, dr, dt4, 1.0)
    torch.cuda.synchronize()
    after = S.to_numpy(n)
    assert ctx.status() & sph.STATUS_NN_RANGE == 0
    t = before["type"][:n0]
    fl = t == cases.FLUID
    ng = t != cases.GHOST
    f64 = lambda a: a.astype(np.float64)
    # references in FP64; the kernel may contract a product into the
    # following add (one rounding instead of two): allow one FP32 ulp
    for d, k in enumerate(("vx", "vy", "vz")):
        xk = "xyz"[d]
        dvv = f64(Y[:, d]) * float(dv)
        vn = f64(before[k][:n0]) + dvv
        xn = f64(before[xk][:n0]) + float(dt4) * 0.5 * (f64(before[k][:n0]) + vn)
        assert np.all(np.abs(f64(after[k][:n0][fl]) - vn[fl]) <= 1.01 * ulp32(vn[fl])), k
        assert np.all(np.abs(f64(after[xk][:n0][fl]) - xn[fl]) <= 2.01 * ulp32(xn[fl])), xk
        vp = vn - 0.25 * dvv
        big = np.maximum(np.abs(vn[fl]), np.abs(vp[fl]))  # vp inherits vn's rounding
        assert np.all(np.abs(f64(after[k + "p"][:n0][fl]) - vp[fl]) <= 2.01 * ulp32(big)), k
        assert np.array_equal(after[k][:n0][~fl], before[k][:n0][~fl])
        assert np.array_equal(after[xk][:n0][~fl], before[xk][:n0][~fl])
    drr = f64(Y[:, 3]) * float(dr)
    rn = f64(before["rho"][:n0]) + drr
    assert np.all(np.abs(f64(after["rho"][:n0][ng]) - rn[ng]) <= 1.01 * ulp32(rn[ng]))
    rp = rn - 0.25 * drr
    big = np.maximum(np.abs(rn[ng]), np.abs(rp[ng]))
    assert np.all(np.abs(f64(after["rhop"][:n0][ng]) - rp[ng]) <= 2.01 * ulp32(big))
    assert np.array_equal(after["rho"][:n0][~ng], before["rho"][:n0][~ng])
    assert np.array_equal(after["rho"][n0:], before["rho"][n0:])
    # with rates: change = dt4 rates + y scale (a product, then an FMA)
    before = after
    rts = (rng.standard_normal((n0, 4)) * [3, 3, 3, 200]).astype(np.float32)
    ctx.nn_apply(S, torch.from_numpy(Y).cuda(), n0, dv, dr, dt4, 1.0,
                 rates=torch.from_numpy(rts).cuda())
    torch.cuda.synchronize()
    after = S.to_numpy(n)
    for d, k in enumerate(("vx", "vy", "vz")):
        inner = f64(before[k][:n0]) + float(dt4) * f64(rts[:, d])  # rounded once first
        vn = inner + f64(Y[:, d]) * float(dv)
        tol = 1.01 * ulp32(vn) + 0.51 * ulp32(inner)
        assert np.all(np.abs(f64(after[k][:n0][fl]) - vn[fl]) <= tol[fl]), k
        assert np.array_equal(after[k][:n0][~fl], before[k][:n0][~fl])
    inner = f64(before["rho"][:n0]) + float(dt4) * f64(rts[:, 3])
    rn = inner + f64(Y[:, 3]) * float(dr)
    tol = 1.01 * ulp32(rn) + 0.51 * ulp32(inner)
    assert np.all(np.abs(f64(after["rho"][:n0][ng]) - rn[ng]) <= tol[ng])
    assert np.array_equal(after["rho"][:n0][~ng], before["rho"][:n0][~ng])
    # carried previous-step differences: prev' = new - (old - prev)
    before = after
    ctx.nn_apply(S, torch.from_numpy(Y).cuda(), n0, dv, dr, dt4, 1.0, carry_prev=True)
    torch.cuda.synchronize()
    after = S.to_numpy(n)
    for k in ("vx", "vy", "vz", "rho"):
        sel = fl if k != "rho" else ng
        diff = f64(before[k][:n0]) - f64(before[k + "p"][:n0])
        want = f64(after[k][:n0]) - diff
        big = np.maximum(np.abs(f64(after[k][:n0])), np.abs(diff))
        assert np.all(np.abs(f64(after[k + "p"][:n0][sel]) - want[sel]) <= 1.01 * ulp32(big[sel])), k
    # a density outside the band raises the status bit
    ctx.nn_apply(S, torch.from_numpy(Y).cuda(), n0, dv, np.float32(50.0), dt4, 0.01)
    assert ctx.status() & sph.STATUS_NN_RANGE


def _advance_pair(case, net, dv=0.02, dr=2.0, dt4=2e-4, residual=False, inv_dt=0.0,
                  carry=False):
    """The unfused chain (features, forward, apply) and the fused advance from
    the same state; returns both states and the unfused outputs."""
    p, n = case.params, case.n
    sc = _scales(p, inv_dt)
    ctx = sph.Context(p, n, sph.FEATURE_SURROGATE)
    ctx.mlp_sync(net)
    cur = sph.DeviceState.from_numpy(case.state)
    U, F = sph.DeviceState.empty(n), sph.DeviceState.empty(n)
    ctx.sort(cur, U, n)
    n0 = ctx.counts()["n_label"][0]
    X = torch.empty(n0, sph.NN_IN, dtype=torch.bfloat16, device="cuda")
    Y = torch.empty(n0, 4, device="cuda")
    R = torch.empty(n0, 4, device="cuda") if residual else None
    ctx.nn_features(U, None, n0, sc, X, rates=R)
    ctx.mlp_forward(net, X, n0, Y)
    ctx.nn_apply(U, Y, n0, dv, dr, dt4, 1.0, rates=R, carry_prev=carry)
    ctx.nn_advance(net, cur, F, n, sc, dv, dr, dt4, 1.0, residual=residual, carry_prev=carry)
    torch.cuda.synchronize()
    return ctx, U, F, X, Y, n0


@pytest.mark.parametrize("residual", [False, True])
@pytest.mark.parametrize("name", ["small_tank", "small_slab", "tank_prev"])
def test_fused_advance_matches_unfused(name, residual):
    case = FEATURE_CASES[name]()
    n = case.n
    announce(f"nn fused vs unfused {name} residual={residual} n={n}")
    net, _ = _random_net(128, case.n, 13, out_gain=50.0)
    prev = name.endswith("prev")
    ctx, U, F, X, Y, n0 = _advance_pair(case, net, residual=residual,
                                        inv_dt=1.0 / 6e-5 if prev else 0.0, carry=prev)
    assert ctx.status() & sph.STATUS_NN_RANGE == 0
    u, f = U.to_numpy(n), F.to_numpy(n)
    assert np.array_equal(u["id"], f["id"])
    for k in sph.F32_FIELDS:
        assert np.array_equal(u[k], f[k]), k
    assert float(Y.abs().max()) > 0.1


def test_judge_sums():
    case = cases.perturb(cases.small_tank(), 8)
    n = case.n
    announce(f"nn judge n={n}")
    net, _ = _random_net(128, case.n, 17, out_gain=50.0)
    ctx, U, F, X, Y, n0 = _advance_pair(case, net)
    Bst = sph.DeviceState.from_numpy(case.state)
    R = sph.DeviceState.empty(n)
    R2 = sph.DeviceState.empty(n)
    ctx.step(Bst, R, n, 0)
    ctx.step(R, R2, n, 1)
    wr = torch.empty(n, dtype=torch.int32, device="cuda")
    wb = torch.empty(n, dtype=torch.int32, device="cuda")
    ctx.nn_index(R2.t["id"], n, wr)
    ctx.nn_index(Bst.t["id"], n, wb)
    m = ctx.nn_judge(F, R2, Bst, wr, wb, n)
    s, r, b = F.to_numpy(n), _by_id(R2.to_numpy(n)), _by_id(Bst.to_numpy(n))
    fl = s["type"] == cases.FLUID
    ids = s["id"][fl]
    g = lambda d, k: d[k][ids].astype(np.float64) if d is not s else s[k][fl].astype(np.float64)
    rs, rr, rb = g(s, "rho"), g(r, "rho"), g(b, "rho")
    want = [np.max(np.abs(rs - rr) / rr), np.sum((rs - rr) ** 2), np.sum((rr - rb) ** 2),
            sum(np.sum((g(s, k) - g(r, k)) ** 2) for k in ("vx", "vy", "vz")),
            sum(np.sum((g(r, k) - g(b, k)) ** 2) for k in ("vx", "vy", "vz")),
            sum(np.sum((g(s, k) - g(r, k)) ** 2) for k in ("x", "y", "z")),
            sum(np.sum((g(r, k) - g(b, k)) ** 2) for k in ("x", "y", "z")), float(fl.sum())]
    assert m[0] == want[0]
    assert np.allclose(m[1:], want[1:], rtol=1e-12, atol=0)


def test_fused_advance_c2_sampled_vs_oracle():
    """The 1.47M-particle workload in the call the surrogate loop makes
    (sph_nn_advance): sampled particles against the oracle's rows and FP64
    network (bfloat16 tensors emulated), applied in FP64."""
    case = cases.perturb(cases.case_c2(), 9)
    p, n = case.params, case.n
    announce(f"nn fused advance c2 n={n}")
    net, arr = _random_net(128, 64, 19, out_gain=50.0)
    sc = _scales(p)
    ctx = sph.Context(p, n, sph.FEATURE_SURROGATE)
    ctx.mlp_sync(net)
    cur = sph.DeviceState.from_numpy(case.state)
    F = sph.DeviceState.empty(n)
    dv, dr, dt4 = np.float32(0.02), np.float32(2.0), np.float32(2e-4)
    ctx.nn_advance(net, cur, F, n, sc, dv, dr, dt4, 1.0, residual=True)
    torch.cuda.synchronize()
    assert ctx.status() & (sph.STATUS_NN_RANGE | sph.STATUS_NONFINITE) == 0
    got = F.to_numpy(n)
    srt = oracle.sort_state(p, case.state)
    assert np.array_equal(got["id"], srt["state"]["id"])
    n0 = int(srt["counts"][0])
    sel = np.sort(np.random.default_rng(5).choice(n0, 4000, replace=False))
    Xo = om.features(p, srt, sel, sc)
    Ro = om.rates(p, srt, sel, sc)
    W, b = _oracle_net(arr)
    Yo, _ = om.forward(W, b, Xo, emulate=True)
    s0 = srt["state"]
    t = s0["type"][sel]
    fl = t == cases.FLUID
    d_rho_gpu = got["rho"][sel].astype(np.float64) - s0["rho"][sel]
    d_rho_ref = Yo[:, 3] * float(dr) + float(dt4) * Ro[:, 3]
    assert relnorm(d_rho_gpu, d_rho_ref) <= 2e-3
    for d, k in enumerate(("vx", "vy", "vz")):
        dv_gpu = got[k][sel][fl].astype(np.float64) - s0[k][sel][fl]
        assert relnorm(dv_gpu, Yo[fl, d] * float(dv) + float(dt4) * Ro[fl, d]) <= 2e-3, k

"""GPU parity of the learned sparse-cell fallback against the MLP reference.

Exact: the training/sparse vertex lists and the BF16 input features.
Within tolerance: the forward output and the training steps' gradients.
The GPU accumulates in FP32 on MFMA, the reference in FP64; the difference of
a pre-activation is ~1e-6 relative, which flips the BF16 rounding of an
activation (2^-8 relative) with probability ~3e-4 per element.  Hence most
outputs agree to ~1e-5 relative and a few percent carry one flipped
activation (effect ~1e-3 of the output scale).  Gradients are sums over the
batch in which flipped activations mostly cancel: measured per parameter
block over four steps of 4096 samples, 4.7e-6 (b3) to 1.1e-5 (W1) relative
in norm; the tests allow 1e-4.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_05942_amd as pf
import synth
from oracle import mlp as om
from synth.mlp_init import init_params
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def _frame(w=480, h=270, frame=0, s=0.04):
    """A scaled frame; s = 0.04 gives cells as populated as s = 0.01 at 1080p."""
    wl = synth.get("hd_1080p_x3")
    f = synth.generate(wl, frame=frame, width=w, height=h)
    f["log2_slots"] = 20
    f["s"] = s
    return wl, f


def _filtered(f, temporal=False):
    """GPU frame (no moving average) with per-vertex counts; oracle beside it."""
    g = to_dev(f)
    n = g["px"].numel()
    flt = pf.FrameFilter(n, f["log2_slots"], temporal=temporal, agg_width=64)
    out = flt.filter(g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], g["valid"], g["r"], g["g"], g["b"],
                     f["cam"], f["s"], f["seed"], with_count=True)
    torch.cuda.synchronize()
    R = oracle.filter_frame({k: (v.cpu() if torch.is_tensor(v) else v) for k, v in f.items()}, temporal=False)
    assert np.array_equal(flt.count[:n].cpu().numpy().view(np.uint32), R.cnt)
    return g, flt, out, R


def _select(flt, n):
    tr = torch.empty(n, dtype=torch.int32, device="cuda")
    sp = torch.empty(n, dtype=torch.int32, device="cuda")
    counts = torch.zeros(2, dtype=torch.int32, device="cuda")
    ws = torch.empty(pf.mlp_select_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    pf.mlp_select(flt.vflags[:n], flt.count[:n], 4, 16, tr, sp, counts, ws)
    torch.cuda.synchronize()
    c = counts.cpu().numpy()
    return tr, sp, counts, int(c[0]), int(c[1])


def test_select_lists_are_exact(gpu):
    wl, f = _frame()
    g, flt, _, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, _, nt, ns = _select(flt, n)
    ok = R.flags == 0
    want_tr = np.nonzero(ok & (R.cnt >= 16))[0]
    want_sp = np.nonzero(ok & (R.cnt < 4))[0]
    assert nt == len(want_tr) and ns == len(want_sp) and nt > 1000 and ns > 1000
    assert np.array_equal(tr[:nt].cpu().numpy(), want_tr)
    assert np.array_equal(sp[:ns].cpu().numpy(), want_sp)
    # one workspace through a sequence of calls: arrays that start one vertex
    # in (not 16-byte aligned: the per-vertex loads instead of the 16-byte
    # ones), ragged and short ranges (one block, a few, 71), the whole frame
    # again, then an empty call
    ws = torch.empty(pf.mlp_select_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    want_t, want_s = ok & (R.cnt >= 16), ok & (R.cnt < 4)
    for lo_v, hi_v in ((1, n), (0, n), (0, 4096), (5, 3 * 4096 + 17), (0, 70 * 4096 + 1000), (3, n), (0, 1)):
        m = hi_v - lo_v
        tr1 = torch.full((m,), -1, dtype=torch.int32, device="cuda")
        sp1 = torch.full((m,), -1, dtype=torch.int32, device="cuda")
        c1 = torch.full((2,), -1, dtype=torch.int32, device="cuda")
        pf.mlp_select(flt.vflags[lo_v:hi_v], flt.count[lo_v:hi_v], 4, 16, tr1, sp1, c1, ws)
        nt1, ns1 = (int(v) for v in c1.cpu().numpy())
        et, es = np.nonzero(want_t[lo_v:hi_v])[0], np.nonzero(want_s[lo_v:hi_v])[0]
        assert (nt1, ns1) == (len(et), len(es)), (lo_v, hi_v)
        assert np.array_equal(tr1[:nt1].cpu().numpy(), et), (lo_v, hi_v)
        assert np.array_equal(sp1[:ns1].cpu().numpy(), es), (lo_v, hi_v)
    # empty input: counts become zero
    counts = torch.full((2,), 7, dtype=torch.int32, device="cuda")
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    pf.mlp_select(torch.empty(0, dtype=torch.uint8, device="cuda"), e, 4, 16, e, e, counts, ws)
    assert counts.cpu().tolist() == [0, 0]
    pf.mlp_select(flt.vflags[:n], flt.count[:n], 4, 16, tr, sp, counts, ws)
    assert counts.cpu().tolist() == [nt, ns]
    assert np.array_equal(tr[:nt].cpu().numpy(), want_tr)
    assert np.array_equal(sp[:ns].cpu().numpy(), want_sp)


def _geo(g, flt, f):
    n = g["px"].numel()
    return pf.geometry(flt.key[:n], g["px"], g["py"], g["pz"], g["nx"], g["ny"], g["nz"], f["cam"])


def _host_geo(f, R, idx):
    pos = np.stack([f["px"].numpy(), f["py"].numpy(), f["pz"].numpy()], 1)[idx]
    nrm = np.stack([f["nx"].numpy(), f["ny"].numpy(), f["nz"].numpy()], 1)[idx]
    return R.key[idx], pos, nrm


def test_features_are_bit_exact(gpu):
    wl, f = _frame()
    g, flt, _, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, _, nt, ns = _select(flt, n)
    idx = torch.cat([tr[:nt], sp[:ns]])
    out = torch.empty((idx.numel(), 80), dtype=torch.int16, device="cuda")
    pf.mlp_features(_geo(g, flt, f), idx, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint16)
    k, pos, nrm = _host_geo(f, R, idx.cpu().numpy())
    want = om.bf16_bits(om.features(k, pos, nrm, f["cam"]))
    assert np.array_equal(got, want), int((got != want).sum())


def test_positional_features_exhaustive(gpu):
    """Every phase the positional encoding can take: the quantised position
    q in [-2^16, 2^16) on all three axes at levels l' = -16, -4, 8, whose 12
    frequencies cover every exponent e = l' - 11 + j from -27 to 8 (the
    phases (2q + 1) 2^e with e < 0 are the ones evaluated with sinpi and
    cospi; e >= 0 gives 0 and +-1).  All 80 inputs of 393,216 keys equal
    the reference's bit for bit."""
    q = np.arange(-65536, 65536, dtype=np.int64)
    keys = []
    for lp in (-16, -4, 8):
        u = (q + 65536).astype(np.uint64)
        keys.append(u | (u << np.uint64(17)) | (u << np.uint64(34)) | np.uint64(lp + 16) << np.uint64(51))
    k = np.concatenate(keys)
    n = k.size
    rng = np.random.default_rng(11)
    pos = rng.uniform(-4, 4, (n, 3)).astype(np.float32)
    nrm = rng.normal(0, 1, (n, 3))
    nrm = (nrm / np.linalg.norm(nrm, axis=1, keepdims=True)).astype(np.float32)
    cam = np.array([0.5, 1.5, -7.0], np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    geo = pf.geometry(dev(k.view(np.int64)), dev(pos[:, 0]), dev(pos[:, 1]), dev(pos[:, 2]), dev(nrm[:, 0]),
                      dev(nrm[:, 1]), dev(nrm[:, 2]), cam)
    idx = torch.arange(n, dtype=torch.int32, device="cuda")
    out = torch.empty((n, 80), dtype=torch.int16, device="cuda")
    pf.mlp_features(geo, idx, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint16)
    want = om.bf16_bits(om.features(k, pos, nrm, cam))
    bad = got != want
    assert not bad.any(), (int(bad.sum()), np.argwhere(bad)[:5].tolist())


def test_inference_matches_reference(gpu):
    wl, f = _frame()
    g, flt, out, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, counts, nt, ns = _select(flt, n)
    net = pf.Mlp(4096)
    w0 = init_params(1902)
    rng = np.random.default_rng(3)
    w0 = (w0 + (rng.normal(0, 0.1, w0.shape) * (w0 != 0))).astype(np.float32)   # make outputs non-trivial
    w0[om.unpack(np.arange(om.N_PARAM))["b1"].astype(int)] = 0.05
    pf.mlp_init(net, w0)
    r, gg, b = (o.clone() for o in out)
    pf.mlp_infer(net, _geo(g, flt, f), sp[:ns], counts, r, gg, b)
    torch.cuda.synchronize()
    idx = sp[:ns].cpu().numpy()
    got = np.stack([r.cpu().numpy(), gg.cpu().numpy(), b.cpu().numpy()], 1)[idx].astype(np.float64)
    k, pos, nrm = _host_geo(f, R, idx)
    want = om.predict(w0.astype(np.float64), om.features(k, pos, nrm, f["cam"]))
    scale = np.abs(want).max()
    assert scale > 0.1
    err = np.abs(got - want) / scale
    assert np.quantile(err, 0.99) < 1e-5 and err.max() < 1e-2, (np.quantile(err, 0.99), err.max())
    # non-sparse vertices are untouched
    mask = np.ones(n, bool); mask[idx] = False
    assert np.array_equal(r.cpu().numpy()[mask], out[0].cpu().numpy()[mask])


def test_one_training_step_matches_reference(gpu):
    wl, f = _frame()
    g, flt, out, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, counts, nt, ns = _select(flt, n)
    batch, seed, lr = 4096, 0x1234_5678_9ABC_DEF0, 1e-3
    net = pf.Mlp(batch)
    w0 = init_params(1902)
    pf.mlp_init(net, w0)
    pf.mlp_train_step(net, flt.cur if flt.temporal else flt.tables[0], _geo(g, flt, f), flt.slot[:n], tr[:nt],
                      counts, batch, seed, lr)
    torch.cuda.synchronize()
    parts = net.partials(batch // 64).cpu().numpy().astype(np.float64)
    g_gpu, loss_gpu = parts[:, :om.N_PARAM].sum(0), parts[:, om.N_PARAM].sum() / (3 * batch)
    assert abs(float(net.loss().cpu()[0]) - loss_gpu) <= 1e-6 * loss_gpu
    # reference: same samples (PCG32 first outputs), targets = oracle cell averages
    u = oracle.pcg32_first(seed, batch).astype(np.uint64)
    pick = (u * np.uint64(nt)) >> np.uint64(32)
    v = np.nonzero((R.flags == 0) & (R.cnt >= 16))[0][pick.astype(np.int64)]
    k, pos, nrm = _host_geo(f, R, v)
    x = om.features(k, pos, nrm, f["cam"])
    t = R.gavg[R.vgroup[v]]
    loss_ref, g_ref = om.loss_and_grad(w0.astype(np.float64), x, t)
    assert abs(loss_gpu - loss_ref) <= 1e-3 * loss_ref, (loss_gpu, loss_ref)
    for name, _ in om.PARAM_SHAPES:
        a, bref = om.unpack(g_gpu)[name], om.unpack(g_ref)[name]
        rel = np.linalg.norm(a - bref) / max(np.linalg.norm(bref), 1e-30)
        assert rel < 1e-4, (name, rel)
    # Adam's first step: w1 = w0 - lr g / (|g| + eps), with the GPU's own gradient
    w1 = net.weights().cpu().numpy().astype(np.float64)
    step = w1 - w0
    assert np.allclose(step, -lr * g_gpu / (np.abs(g_gpu) + 1e-8), atol=2e-7)
    # ...and it equals the reference step on clearly non-zero gradient elements
    w_ref, _, _ = om.adam_step(w0, np.zeros_like(w0), np.zeros_like(w0), g_ref, 1, lr)
    big = np.abs(g_ref) > 0.05 * np.abs(g_ref).max()
    assert big.sum() > 100 and (np.sign(g_gpu[big]) == np.sign(g_ref[big])).mean() > 0.999
    same = big & (np.sign(g_gpu) == np.sign(g_ref))
    assert np.allclose(w1[same], w_ref[same], atol=2e-7)
    wb = net.weights_bf16().cpu().numpy().view(np.uint16)
    assert np.array_equal(wb, om.bf16_bits(w1.astype(np.float32)))


def test_training_is_deterministic(gpu):
    wl, f = _frame(320, 180)
    g, flt, out, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, counts, nt, ns = _select(flt, n)
    ws = []
    for _ in range(2):
        net = pf.Mlp(2048)
        pf.mlp_init(net, init_params(5))
        for s in range(3):
            pf.mlp_train_step(net, flt.tables[0], _geo(g, flt, f), flt.slot[:n], tr[:nt], counts, 2048, 77 + s, 1e-3)
        torch.cuda.synchronize()
        ws.append(net.weights().cpu().numpy())
    assert np.array_equal(ws[0], ws[1])


def test_learned_fallback_beats_the_plain_average_on_sparse_cells(gpu):
    """16 frames of the orbiting 1080p x3 workload with the moving average:
    training on cells with >= 16 samples and predicting cells with < 4 must
    lower the error against the noise-free radiance on those sparse-cell
    vertices compared with the filter alone."""
    wl = synth.get("hd_1080p_x3_mlp")
    W, H = 1920, 1080
    n = W * H * 3
    fb = pf.MlpFallback(n, init_params(1902), batch=16384, steps=4, lr=1e-3)
    with_mlp = pf.FrameFilter(n, 22, temporal=True, alpha_old=wl.alpha_old, agg_width=64, mlp=fb)
    plain = pf.FrameFilter(n, 22, temporal=True, alpha_old=wl.alpha_old, agg_width=64)
    for frame in range(16):
        f = synth.generate(wl, frame=frame, width=W, height=H, device="cuda")
        args = (f["px"], f["py"], f["pz"], f["nx"], f["ny"], f["nz"], f["valid"], f["r"], f["g"], f["b"], f["cam"],
                f["s"], f["seed"])
        o_mlp = with_mlp.filter(*args)
        o_plain = plain.filter(*args, with_count=True)
    torch.cuda.synchronize()
    sparse = (plain.vflags[:n] == 0) & (plain.count[:n] < 4)
    truth = f["truth"]
    def rmse(o, m):
        return float(torch.sqrt(((torch.stack(o, 1)[m] - truth[m]) ** 2).mean()))
    e_mlp, e_plain = rmse(o_mlp, sparse), rmse(o_plain, sparse)
    valid = f["valid"].bool()
    print(f"sparse vertices {int(sparse.sum())}: rmse plain {e_plain:.4f} mlp {e_mlp:.4f}; "
          f"all valid: plain {rmse(o_plain, valid):.4f} mlp {rmse(o_mlp, valid):.4f}; "
          f"loss {float(fb.net.loss().cpu()[0]):.5f}")
    assert int(sparse.sum()) > 1000
    assert e_mlp < 0.8 * e_plain
    assert rmse(o_mlp, valid) < rmse(o_plain, valid)


def test_four_adam_steps_match_the_reference(gpu):
    """Four consecutive training steps on one frame.  At every step the GPU's
    gradient (its per-workgroup partials) is compared with the reference
    gradient at the GPU's current weights, and the GPU's Adam update (weights
    and both moments) with the reference Adam step fed that gradient, which
    checks the bias corrections 1 / (1 - beta^t) for t = 1..4 and the moment
    recurrences after the first step."""
    wl, f = _frame()
    g, flt, out, R = _filtered(f)
    n = g["px"].numel()
    tr, sp, counts, nt, ns = _select(flt, n)
    batch, lr = 4096, 1e-3
    net = pf.Mlp(batch)
    w = init_params(1902).astype(np.float32)
    pf.mlp_init(net, w)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    geo = _geo(g, flt, f)
    train_v = np.nonzero((R.flags == 0) & (R.cnt >= 16))[0]
    worst = {}
    for step in range(1, 5):
        seed = 0x9E37_79B9_7F4A_7C15 + step
        pf.mlp_train_step(net, flt.tables[0], geo, flt.slot[:n], tr[:nt], counts, batch, seed, lr, step=step)
        torch.cuda.synchronize()
        parts = net.partials(batch // 64).cpu().numpy().astype(np.float64)
        g_gpu = parts[:, :om.N_PARAM].sum(0)
        # reference gradient at the weights this step started from
        u = oracle.pcg32_first(seed, batch).astype(np.uint64)
        vtx = train_v[((u * np.uint64(nt)) >> np.uint64(32)).astype(np.int64)]
        k, pos, nrm = _host_geo(f, R, vtx)
        _, g_ref = om.loss_and_grad(w.astype(np.float64), om.features(k, pos, nrm, f["cam"]), R.gavg[R.vgroup[vtx]])
        for name, _ in om.PARAM_SHAPES:
            a, b = om.unpack(g_gpu)[name], om.unpack(g_ref)[name]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            worst[name] = max(worst.get(name, 0.0), rel)
        # the reference Adam step fed the GPU's gradient
        w_ref, m_ref, v_ref = om.adam_step(w, m, v, g_gpu, step, lr)
        w_gpu = net.weights().cpu().numpy()
        m_gpu, v_gpu = (x.cpu().numpy() for x in net.moments())
        assert np.allclose(m_gpu, m_ref, rtol=1e-5, atol=1e-6 * np.abs(m_ref).max()), step
        assert np.allclose(v_gpu, v_ref, rtol=1e-5, atol=1e-6 * np.abs(v_ref).max()), step
        d_gpu, d_ref = w_gpu.astype(np.float64) - w, w_ref.astype(np.float64) - w
        # elements whose second moment is not at the level of the summation
        # error of the gradient: the steps agree to 1e-4 of lr
        firm = np.sqrt(v_ref / (1 - 0.999 ** step)) > 1e-4 * np.sqrt(v_ref.max())
        assert firm.sum() > 0.5 * firm.size
        assert np.abs(d_gpu - d_ref)[firm].max() <= 1e-4 * lr + 2 ** -23 * np.abs(w)[firm].max(), step
        # every element moves by at most Adam's bound lr * (1 - b1) / sqrt(1 - b2) per step (and at step 1 by lr)
        assert np.abs(d_gpu).max() <= lr * 3.2 + 1e-7
        wb = net.weights_bf16().cpu().numpy().view(np.uint16)
        assert np.array_equal(wb, om.bf16_bits(w_gpu))
        w, m, v = w_gpu, m_gpu, v_gpu
    print("worst gradient relative error per block over 4 steps:",
          {k: float(f"{x:.2e}") for k, x in worst.items()})
    assert all(x < 1e-4 for x in worst.values()), worst

"""GPU differentiable path: FP64 float-path forward against the C oracle, and the
hand-written backward against the torch-FP64 gradient oracle."""
import numpy as np
import pytest
import torch

from _common import DISP_TOL, PASS_FRAC, oracle_params, parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2205_03133_amd import bdis
    bdis.lib()
    return bdis


def _pair(h, w, seed=0):
    from paper_2205_03133_amd.synth import make_pair
    left, right, gt, valid = make_pair(4, seed, quantize=False)
    return (np.ascontiguousarray(left[:h, :w]).astype(np.float32),
            np.ascontiguousarray(right[:h, :w]).astype(np.float32), gt[:h, :w], valid[:h, :w])


def _fparams(B, **kw):
    base = dict(levels=3, patch=8, stride=4, iters=8, float_pyramid=1, variance=1)
    base.update(kw)
    return B.params(**base)


@pytest.mark.parametrize("shape,kw", [((96, 160), {}), ((480, 640), dict(levels=4, variance=0)),
                                      ((101, 133), dict(patch=7, stride=3, sigma_r_dynamic=0, sigma_r=6.0)),
                                      ((120, 200), dict(levels=4, finest_level=1))])
def test_float_forward_parity(B, oracle, shape, kw):
    h, w = shape
    left, right, _, _ = _pair(h, w)
    p = _fparams(B, **kw)
    print(f"[gpu] float path {w}x{h} {kw}", flush=True)
    ctx = B.Context(p, w, h, train=True)
    out = ctx.compute_f32(torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda())
    torch.cuda.synchronize()
    r = oracle.compute(left.astype(np.float64), right.astype(np.float64), oracle_params(oracle, p))
    st = parity(out["disp"].cpu().numpy(), r["disp"], DISP_TOL)
    print(f"  disparity frac={st['frac']:.6f} max={st['max_err']:.3g} mask={st['mask_mismatch']}", flush=True)
    assert st["frac"] >= PASS_FRAC
    if p.variance:
        sv = parity(out["var"].cpu().numpy(), r["var"], 1e-3, rel=True)
        print(f"  variance frac={sv['frac']:.6f}", flush=True)
        assert sv["frac"] >= PASS_FRAC
    ctx.close()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("shape,kw", [((48, 80), dict(levels=1, iters=6)),
                                      ((48, 80), dict(levels=2, iters=6)),
                                      ((64, 112), dict(levels=3, iters=8, sigma_r_dynamic=0, sigma_r=6.0)),
                                      ((96, 160), dict(levels=3, iters=8))])
def test_backward_matches_gradient_oracle(B, oracle, shape, kw):
    from oracle import grad_ref as GR
    h, w = shape
    left, right, _, _ = _pair(h, w, seed=1)
    p = _fparams(B, **kw)
    rng = np.random.default_rng(2)
    v_disp = rng.standard_normal((h, w))
    v_var = 0.01 * rng.standard_normal((h, w))
    print(f"[gpu] backward {w}x{h} {kw}", flush=True)
    ctx = B.Context(p, w, h, train=True)
    lt, rt = torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda()
    out = ctx.compute_f32(lt, rt)
    gl, gr, gh = ctx.backward(torch.from_numpy(v_disp.astype(np.float32)).cuda(),
                              torch.from_numpy(v_var.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    ref = GR.loss_and_grads(left.astype(np.float64), right.astype(np.float64), oracle_params(oracle, p),
                            v_disp.astype(np.float32).astype(np.float64),
                            v_var.astype(np.float32).astype(np.float64))
    gl, gr, gh = gl.cpu().numpy(), gr.cpu().numpy(), gh.cpu().numpy()
    e_l, e_r = _rel(gl, ref["left"]), _rel(gr, ref["right"])
    hyp = np.array([ref["sigma_s"], ref["sigma_r"]] + list(ref["omega"]))
    print(f"  rel err: left {e_l:.2e} right {e_r:.2e}; hyper gpu {gh} oracle {hyp}", flush=True)
    assert e_l <= 1e-3 and e_r <= 1e-3
    np.testing.assert_allclose(gh, hyp, rtol=1e-3, atol=1e-6 * np.abs(hyp).max())
    ctx.close()


def _backward_vs_oracle(B, oracle, pairs, kw, seed=2):
    """GPU backward of a batch of float pairs against the FP64 gradient oracle,
    pair by pair (image gradients) and summed (hyper-gradients)."""
    from oracle import grad_ref as GR
    h, w = pairs[0][0].shape
    p = _fparams(B, **kw)
    n = len(pairs)
    rng = np.random.default_rng(seed)
    vd = [rng.standard_normal((h, w)).astype(np.float32) for _ in range(n)]
    vv = [(0.01 * rng.standard_normal((h, w))).astype(np.float32) for _ in range(n)] if p.variance else None
    ctx = B.Context(p, w, h, max_batch=n, train=True)
    L = torch.stack([torch.from_numpy(q[0]) for q in pairs]).cuda()
    R = torch.stack([torch.from_numpy(q[1]) for q in pairs]).cuda()
    ctx.compute_f32(L, R)
    gl, gr, gh = ctx.backward(torch.from_numpy(np.stack(vd)).cuda(),
                              torch.from_numpy(np.stack(vv)).cuda() if vv is not None else None)
    torch.cuda.synchronize()
    gl, gr, gh = gl.cpu().numpy(), gr.cpu().numpy(), gh.cpu().numpy()
    hyp = 0.0
    for b in range(n):
        ref = GR.loss_and_grads(pairs[b][0].astype(np.float64), pairs[b][1].astype(np.float64),
                                oracle_params(oracle, p), vd[b].astype(np.float64),
                                vv[b].astype(np.float64) if vv is not None else None)
        e_l, e_r = _rel(gl[b], ref["left"]), _rel(gr[b], ref["right"])
        print(f"  pair {b}: rel err left {e_l:.2e} right {e_r:.2e}", flush=True)
        assert e_l <= 1e-3 and e_r <= 1e-3
        hyp = hyp + np.array([ref["sigma_s"], ref["sigma_r"]] + list(ref["omega"]))
    print(f"  hyper gpu {gh} oracle {hyp}", flush=True)
    np.testing.assert_allclose(gh, hyp, rtol=1e-3, atol=1e-6 * np.abs(hyp).max())
    ctx.close()


@pytest.mark.parametrize("n", [1, 2])
def test_backward_full_size_differentiation_workload(B, oracle, n):
    """The differentiation workload's shape: 640x480 float pairs, 4 levels, 8x8
    patches, stride 4, K = 8 unrolled; one pair and a batch of two."""
    pairs = [_pair(480, 640, seed=10 + b) for b in range(n)]
    print(f"[gpu] backward 640x480 L4 P8 S4 K8, batch {n}", flush=True)
    _backward_vs_oracle(B, oracle, pairs, dict(levels=4, iters=8, variance=0))


def test_backward_untiled_search_adjoint(B, oracle):
    """Patch 16 at stride 10: the search adjoint's LDS accumulation tiles do not
    fit, so every scatter of that kernel goes straight to HBM."""
    print("[gpu] backward 160x96 L2 P16 S10 K6 (untiled search adjoint)", flush=True)
    _backward_vs_oracle(B, oracle, [_pair(96, 160, seed=4)], dict(levels=2, patch=16, stride=10, iters=6))


def test_autograd_rejects_stale_node(B):
    """Two forwards on one context, then backward of the first: the context keeps
    only the latest call's saved state, so the stale node raises instead of
    returning the second call's gradients."""
    h, w = 64, 96
    left, right, _, _ = _pair(h, w, seed=3)
    ctx = B.Context(_fparams(B, levels=2, iters=6), w, h, train=True)
    fn = B.bdis_function()
    ss = torch.tensor(4.0, dtype=torch.float64, requires_grad=True)
    sr = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    om = torch.tensor([1.0, 2.0], dtype=torch.float64, requires_grad=True)
    print("[gpu] autograd stale node", flush=True)
    lt = torch.from_numpy(left).cuda().requires_grad_(True)
    d1, _ = fn.apply(lt, torch.from_numpy(right).cuda(), ss, sr, om, ctx)
    d2, _ = fn.apply(lt, torch.from_numpy(left).cuda(), ss, sr, om, ctx)
    with pytest.raises(RuntimeError, match="another forward"):
        torch.nan_to_num(d1).sum().backward()
    torch.nan_to_num(d2).sum().backward()  # the latest node still works
    torch.cuda.synchronize()
    assert torch.isfinite(lt.grad).all()
    ctx.close()


def test_repeated_backward_starts_from_cleared_adjoints(B):
    """Backward twice after one forward, and again after a second forward on
    another pair: each call clears its adjoint state first, so repeated calls
    agree (to the rounding of their FP64 atomics) and follow the new pair."""
    h, w = 80, 128
    p = _fparams(B, levels=3, iters=6)
    ctx = B.Context(p, w, h, train=True)
    g = torch.randn((h, w), generator=torch.Generator().manual_seed(1)).cuda()
    res = []
    for seed in (5, 5, 6):
        left, right, _, _ = _pair(h, w, seed=seed)
        print(f"[gpu] backward after forward of pair {seed}", flush=True)
        ctx.compute_f32(torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda())
        gl, gr, gh = ctx.backward(g)
        gl2, gr2, gh2 = ctx.backward(g)
        torch.cuda.synchronize()
        for x, y in ((gl, gl2), (gr, gr2), (gh, gh2)):
            assert torch.allclose(x, y, rtol=1e-9, atol=1e-12)
        res.append((gl.clone(), gr.clone(), gh.clone()))
    for x, y in zip(res[0], res[1]):
        assert torch.allclose(x, y, rtol=1e-9, atol=1e-12)
    assert not torch.allclose(res[0][0], res[2][0])
    ctx.close()


def test_backward_batch_equals_single(B):
    h, w = 64, 96
    p = _fparams(B, levels=2, iters=6)
    pairs = [_pair(h, w, seed=s) for s in range(3)]
    L = torch.stack([torch.from_numpy(q[0]) for q in pairs]).cuda()
    R = torch.stack([torch.from_numpy(q[1]) for q in pairs]).cuda()
    g = torch.randn((3, h, w), generator=torch.Generator().manual_seed(0)).cuda()
    print("[gpu] backward batch of 3 vs single", flush=True)
    ctx = B.Context(p, w, h, max_batch=3, train=True)
    ctx.compute_f32(L, R)
    gl, gr, gh = ctx.backward(g)
    torch.cuda.synchronize()
    tot = torch.zeros_like(gh)
    for b in range(3):
        one = B.Context(p, w, h, train=True)
        one.compute_f32(L[b], R[b])
        l1, r1, h1 = one.backward(g[b])
        torch.cuda.synchronize()
        assert torch.allclose(l1[0], gl[b], rtol=1e-5, atol=1e-7)
        assert torch.allclose(r1[0], gr[b], rtol=1e-5, atol=1e-7)
        tot += h1
        one.close()
    assert torch.allclose(tot, gh, rtol=1e-9, atol=1e-12)
    ctx.close()


def test_autograd_function(B):
    h, w = 64, 96
    left, right, gt, valid = _pair(h, w, seed=3)
    p = _fparams(B, levels=2, iters=6)
    ctx = B.Context(p, w, h, train=True)
    fn = B.bdis_function()
    lt = torch.from_numpy(left).cuda().requires_grad_(True)
    rt = torch.from_numpy(right).cuda().requires_grad_(True)
    ss = torch.tensor(4.0, dtype=torch.float64, requires_grad=True)
    sr = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    om = torch.tensor([1.0, 2.0], dtype=torch.float64, requires_grad=True)
    print("[gpu] autograd function", flush=True)
    disp, var = fn.apply(lt, rt, ss, sr, om, ctx)
    ok = torch.isfinite(disp)
    loss = (disp[ok] ** 2).sum() + var[ok].sum()
    loss.backward()
    torch.cuda.synchronize()
    # the same gradient straight through the context
    ctx2 = B.Context(p, w, h, train=True)
    out = ctx2.compute_f32(lt.detach(), rt.detach())
    gd = torch.where(torch.isfinite(out["disp"]), 2 * out["disp"], torch.zeros_like(out["disp"]))
    gv = torch.where(torch.isfinite(out["disp"]), torch.ones_like(out["disp"]), torch.zeros_like(out["disp"]))
    gl, gr, gh = ctx2.backward(gd, gv)
    torch.cuda.synchronize()
    assert torch.allclose(lt.grad, gl[0], rtol=1e-5, atol=1e-6)
    assert torch.allclose(rt.grad, gr[0], rtol=1e-5, atol=1e-6)
    assert float(ss.grad) == pytest.approx(float(gh[0]), rel=1e-9, abs=1e-9)
    assert float(sr.grad) == pytest.approx(float(gh[1]), rel=1e-9, abs=1e-9)
    assert np.allclose(om.grad.cpu().numpy(), gh[2:4].cpu().numpy(), rtol=1e-9, atol=1e-9)
    ctx.close()
    ctx2.close()


def test_hyperparameter_tuning_reduces_error(B):
    """A few gradient steps on (sigma_s, alpha_r, omega) lower the masked squared
    disparity error against the synthetic ground truth."""
    h, w = 240, 320
    from paper_2205_03133_amd.synth import make_pair
    left, right, gt, valid = make_pair(4, 5, quantize=False)
    left = np.ascontiguousarray(left[:h, :w]).astype(np.float32)
    right = np.ascontiguousarray(right[:h, :w]).astype(np.float32)
    gt_t = torch.from_numpy(gt[:h, :w]).cuda()
    vm = torch.from_numpy(valid[:h, :w]).cuda()
    p = _fparams(B, levels=3, iters=8, variance=0)
    ctx = B.Context(p, w, h, train=True)
    fn = B.bdis_function()
    lt, rt = torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda()
    log_ss = torch.tensor(np.log(4.0), dtype=torch.float64, requires_grad=True)
    log_sr = torch.tensor(0.0, dtype=torch.float64, requires_grad=True)
    log_om = torch.tensor(np.log([1.0, 2.0, 4.0]), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([log_ss, log_sr, log_om], lr=0.1)
    losses = []
    print("[gpu] hyperparameter tuning demo 320x240", flush=True)
    for it in range(8):
        opt.zero_grad()
        disp, _ = fn.apply(lt, rt, log_ss.exp(), log_sr.exp(), log_om.exp(), ctx)
        ok = torch.isfinite(disp) & vm
        err = (disp - gt_t)[ok]
        loss = torch.nn.functional.smooth_l1_loss(err, torch.zeros_like(err), beta=1.0)
        loss.backward()
        opt.step()
        losses.append(float(loss))
    print("  losses", [round(x, 4) for x in losses], flush=True)
    assert min(losses[1:]) < losses[0]
    ctx.close()


def test_backward_needs_finest_level_zero(B):
    h, w = 64, 96
    left, right, _, _ = _pair(h, w)
    p = _fparams(B, levels=3, finest_level=1)
    ctx = B.Context(p, w, h, train=True)
    ctx.compute_f32(torch.from_numpy(left).cuda(), torch.from_numpy(right).cuda())
    with pytest.raises(B.BdisError):
        ctx.backward(torch.zeros((h, w), device="cuda"))
    ctx.close()


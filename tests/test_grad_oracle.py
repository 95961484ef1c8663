"""Pins of the gradient oracle (torch FP64 autograd, CPU).

Its forward must equal the C oracle's float path, and its gradient must equal
central finite differences of the C oracle wherever the perturbed runs take
the same discrete decisions as the base run (equal decision hashes).
"""
import numpy as np
import pytest
import torch

from oracle import grad_ref as GR


def _pair(h=64, w=112, seed=0):
    from paper_2205_03133_amd.synth import make_pair
    left, right, _, _ = make_pair(4, seed, quantize=False)
    return np.ascontiguousarray(left[:h, :w]), np.ascontiguousarray(right[:h, :w])


def _params(oracle, **kw):
    base = dict(levels=3, patch=8, stride=4, iters=8, float_pyramid=1, variance=1)
    base.update(kw)
    return oracle.default_params(**base)


@pytest.mark.parametrize("kw", [dict(), dict(sigma_r_dynamic=0, sigma_r=6.0), dict(variance=0, levels=2),
                                dict(patch=6, stride=2, iters=5)])
def test_forward_equals_c_oracle(oracle, kw):
    left, right = _pair()
    p = _params(oracle, **kw)
    c = oracle.compute(left, right, p)
    ss, sr, om = GR.hyper_tensors(p, requires_grad=False)
    o = GR.forward(torch.tensor(left), torch.tensor(right), p, ss, sr, om)
    d = o["disp"].numpy()
    assert np.array_equal(np.isfinite(d), np.isfinite(c["disp"]))
    ok = np.isfinite(d)
    np.testing.assert_allclose(d[ok], c["disp"][ok], rtol=0, atol=1e-10)
    np.testing.assert_allclose(o["conf"].numpy(), c["conf"], rtol=0, atol=1e-12)
    if p["variance"]:
        np.testing.assert_allclose(o["var"].numpy()[ok], c["var"][ok], rtol=1e-10)


def _c_loss(oracle, left, right, p, v_disp, v_var):
    out = oracle.compute(left, right, p, trace=True)
    ok = np.isfinite(out["disp"])
    loss = float((v_disp[ok] * out["disp"][ok]).sum())
    if v_var is not None:
        loss += float((v_var[ok] * out["var"][ok]).sum())
    return loss, out["trace"].decision_hash()


def test_gradient_matches_finite_differences(oracle):
    left, right = _pair(48, 80, seed=1)
    p = _params(oracle, levels=2, iters=6)
    rng = np.random.default_rng(0)
    v_disp = rng.standard_normal(left.shape)
    v_var = 0.01 * rng.standard_normal(left.shape)
    g = GR.loss_and_grads(left, right, p, v_disp, v_var)
    base_loss, base_hash = _c_loss(oracle, left, right, p, v_disp, v_var)
    assert abs(base_loss - g["loss"]) <= 1e-8 * max(1.0, abs(base_loss))
    checked = 0
    # image directions
    h = 1e-7
    for k in range(6):
        dl = rng.standard_normal(left.shape)
        dr = rng.standard_normal(left.shape)
        lp, hp = _c_loss(oracle, left + h * dl, right + h * dr, p, v_disp, v_var)
        lm, hm = _c_loss(oracle, left - h * dl, right - h * dr, p, v_disp, v_var)
        if not (hp == hm == base_hash):
            continue
        fd = (lp - lm) / (2 * h)
        an = float((g["left"] * dl).sum() + (g["right"] * dr).sum())
        assert fd == pytest.approx(an, rel=2e-4, abs=1e-5), (k, fd, an)
        checked += 1
    assert checked >= 3
    # hyperparameters
    hh = 1e-6
    for name, idx in [("sigma_s", None), ("sigma_r", None), ("omega", 0), ("omega", 1)]:
        pp, pm = dict(p), dict(p)
        if name == "omega":
            lw = list(p["level_weight"])
            lw_p, lw_m = list(lw), list(lw)
            lw_p[idx] += hh
            lw_m[idx] -= hh
            pp["level_weight"], pm["level_weight"] = lw_p, lw_m
            an = float(g["omega"][idx])
        else:
            pp[name] = p[name] + hh
            pm[name] = p[name] - hh
            an = g[name]
        lp, hp = _c_loss(oracle, left, right, pp, v_disp, v_var)
        lm, hm = _c_loss(oracle, left, right, pm, v_disp, v_var)
        if not (hp == hm == base_hash):
            continue
        fd = (lp - lm) / (2 * hh)
        assert fd == pytest.approx(an, rel=2e-4, abs=1e-5), (name, idx, fd, an)
        checked += 1
    assert checked >= 6


def test_gradient_closed_form_posterior_scale(oracle):
    """Row-linear pair, one level, fixed sigma_r: every patch has SSD(d) = H d^2, so
    post = 1/sum_d exp(-H d^2 / tau) and d post / d sigma_r has a closed form; the
    confidence is the mask-weighted average of Gamma_0 * post = post."""
    h, w, P, S = 24, 64, 8, 4
    alpha = 0.8 + 0.05 * np.arange(h)
    xs = np.arange(w, dtype=np.float64)
    left = alpha[:, None] * xs[None, :] + 20.0
    right = alpha[:, None] * (xs[None, :] + 0.6) + 20.0
    p = oracle.default_params(levels=1, patch=P, stride=S, iters=3, float_pyramid=1, sigma_r_dynamic=0,
                              sigma_r=3.0, variance=0)
    lt = torch.tensor(left, dtype=GR.DT)
    rt = torch.tensor(right, dtype=GR.DT)
    ss, sr, om = GR.hyper_tensors(p)
    out = GR.forward(lt, rt, p, ss, sr, om)
    lv = out["levels"][0]
    # pick interior patches (exact quadratic SSD)
    ox = torch.tensor([min(i * S, w - P) for i in range((w - P + S - 1) // S + 1)])
    oy = torch.tensor([min(j * S, h - P) for j in range((h - P + S - 1) // S + 1)])
    nx = len(ox)
    k = 1 * nx + 2  # row 1, column 2: away from the borders
    post = lv["post"][k]
    post.backward()
    Hk = float(lv["ssd"][k, 4].detach())  # SSD(+1) = H
    tau = 2 * 3.0 ** 2 * 25
    d2 = np.array([1.0, 0.25, 0.0, 0.25, 1.0])
    e = np.exp(-Hk * d2 / tau)
    post_cf = 1.0 / e.sum()
    # d post / d tau = -post^2 * sum(e * H d^2 / tau^2); d tau / d sigma_r = 4 sigma_r s^2
    dpost_dtau = -post_cf ** 2 * (e * Hk * d2 / tau ** 2).sum()
    assert float(post) == pytest.approx(post_cf, rel=1e-12)
    assert float(sr.grad) == pytest.approx(dpost_dtau * 4 * 3.0 * 25, rel=1e-9)

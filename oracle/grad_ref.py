"""Gradient oracle: the float path of the BDIS hot path in plain PyTorch FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (imported by the test-suite).  It re-implements the
same steps and readings as the C oracle (``bdis_ref.c``) with differentiable
tensor operations, so autograd gives the gradient of any loss of the outputs
with respect to both images and the hyperparameters (mixture sigma_s,
photometric sigma_r or its scale alpha_r, level weights omega_n).  Discrete
decisions (unit cells, the search-threshold reset, acceptance, holes,
variance-fit outcomes) are taken on values and carry no gradient, as the
method's outputs are piecewise smooth in its inputs.

Its forward is checked against the C oracle, and its gradient against
central finite differences of the C oracle, in the tests.
"""
from __future__ import annotations

import math

import torch
import torch.nn.functional as F

DT = torch.float64
OFFSETS = (-1.0, -0.5, 0.0, 0.5, 1.0)
EPS_H = 1e-3
EPS_SIGMA = 1e-6
NWIN = 5


def _pyr_down(img):
    """Binomial [1 4 6 4 1]/16 (separable), reflect-101 borders, even samples (Sec. III-B)."""
    k1 = torch.tensor([1.0, 4.0, 6.0, 4.0, 1.0], dtype=DT)
    k2 = (k1[:, None] * k1[None, :] / 256.0)[None, None]
    x = F.pad(img[None, None], (2, 2, 2, 2), mode="reflect")
    y = F.conv2d(x, k2)[0, 0]
    return y[::2, ::2]


def _sobel_x(img):
    """Sobel-x / 8 with reflect-101 borders (template gradient, Sec. III-A)."""
    k = torch.tensor([[-1.0, 0.0, 1.0], [-2.0, 0.0, 2.0], [-1.0, 0.0, 1.0]], dtype=DT)[None, None] / 8.0
    x = F.pad(img[None, None], (1, 1, 1, 1), mode="reflect")
    return F.conv2d(x, k)[0, 0]


def _grid(n, P, S):
    cnt = (n - P + S - 1) // S + 1
    return torch.tensor([min(i * S, n - P) for i in range(cnt)], dtype=torch.long)


def _bilinear(m, x, y):
    """Bilinear samples of map m at (x, y) (constant positions), indices clamped."""
    h, w = m.shape
    x0 = torch.floor(x)
    y0 = torch.floor(y)
    ax, ay = x - x0, y - y0
    x0i, y0i = x0.long(), y0.long()
    xa, xb = x0i.clamp(0, w - 1), (x0i + 1).clamp(0, w - 1)
    ya, yb = y0i.clamp(0, h - 1), (y0i + 1).clamp(0, h - 1)
    top = (1 - ax) * m[ya, xa] + ax * m[ya, xb]
    bot = (1 - ax) * m[yb, xa] + ax * m[yb, xb]
    return (1 - ay) * top + ay * bot


def _warp(R, Y, X, u):
    """Linear warp of the right level at X + u (rows Y), indices clamped (Eq. 1)."""
    w = R.shape[1]
    m = torch.floor(u).detach()
    f = (u - m)[:, None, None]
    mi = m.long()[:, None, None]
    a = R[Y, (X + mi).clamp(0, w - 1)]
    b = R[Y, (X + mi + 1).clamp(0, w - 1)]
    return (1 - f) * a + f * b


def mask(P, sigma_s):
    """Spatial mixture mask M[b, a] = sum over patch pixels of exp(-d^2 / (2 sigma_s^2)) (Eq. 9)."""
    ar = torch.arange(P, dtype=DT)
    d1 = (ar[:, None] - ar[None, :]) ** 2          # (a, c)
    e = torch.exp(-(d1[:, None, :, None] + d1[None, :, None, :]) / (2 * sigma_s * sigma_s))  # (b, a, d, c)
    return e.sum((2, 3))


def forward(left, right, params, sigma_s, sigma_r, omega):
    """Float-path forward.  left/right: (H, W) float64 tensors; sigma_s, sigma_r:
    0-d tensors; omega: (L,) tensor.  Returns dict(disp, var, conf, levels)."""
    L = params["levels"]
    f_lv = params["finest_level"]
    P, S, K = params["patch"], params["stride"], params["iters"]
    gamma_valid = params["valid_ratio"]
    assert f_lv == 0
    imgs_l, imgs_r = [left], [right]
    for _ in range(1, L):
        imgs_l.append(_pyr_down(imgs_l[-1]))
        imgs_r.append(_pyr_down(imgs_r[-1]))
    grads = [_sobel_x(x) for x in imgs_l]
    M = mask(P, sigma_s)
    sfail = params["var_fail_sigma"] if params["var_fail_sigma"] > 0 else float(P)
    sfail2 = sfail * sfail
    wsum = omega[f_lv:L].sum()
    ar = torch.arange(P)
    par_u = par_q = None
    out = {}
    trace = []
    for n in range(L - 1, f_lv - 1, -1):
        Lv, Rv, Gv = imgs_l[n], imgs_r[n], grads[n]
        h, w = Lv.shape
        ox, oy = _grid(w, P, S), _grid(h, P, S)
        nx, ny = len(ox), len(oy)
        OX = ox[None, :].expand(ny, nx).reshape(-1)
        OY = oy[:, None].expand(ny, nx).reshape(-1)
        X = OX[:, None, None] + ar[None, None, :]
        Y = OY[:, None, None] + ar[None, :, None]
        T = Lv[Y, X]
        G = Gv[Y, X]
        J = G - G.mean((1, 2), keepdim=True)
        H = (J * J).sum((1, 2))
        if par_u is not None:
            cx = (OX.to(DT) + 0.5 * (P - 1)) * 0.5
            cy = (OY.to(DT) + 0.5 * (P - 1)) * 0.5
            u0 = 2.0 * _bilinear(par_u, cx, cy)
            pipar = _bilinear(par_q, cx, cy)
        else:
            u0 = torch.zeros(nx * ny, dtype=DT)
            pipar = torch.zeros(nx * ny, dtype=DT)
        inv = (H >= EPS_H).detach()
        Hs = torch.where(inv, H, torch.ones_like(H))
        u = u0
        for _ in range(K):
            Iw = _warp(Rv, Y, X, u)
            b = (J * (Iw - T)).sum((1, 2))
            u = torch.where(inv, u - b / Hs, u)
        reset = (torch.abs(u - u0) > P).detach()
        u = torch.where(reset, u0, u)
        ssd = []
        for d in OFFSETS:
            e = _warp(Rv, Y, X, u + d) - T
            ssd.append(((e - e.mean((1, 2), keepdim=True)) ** 2).sum((1, 2)))
        ssd = torch.stack(ssd, 1)
        xr = X.to(DT) + u.detach()[:, None, None]          # (patches, 1, P): one row of columns
        inb = ((xr >= 0) & (xr <= w - 1)).sum((1, 2)).to(DT) * P
        rho = inb / (P * P)
        acc = ((ssd[:, 2:3] <= ssd).all(1) & (rho >= gamma_valid)).detach()
        nacc = int(acc.sum())
        if params["sigma_r_dynamic"]:
            pooled = ssd[:, 2][acc].sum() / (nacc * P * P) if nacc > 0 else torch.zeros((), dtype=DT)
            big = bool(pooled.detach() > EPS_SIGMA)
            sr2 = sigma_r * sigma_r * (pooled if big else torch.full((), EPS_SIGMA, dtype=DT))
        else:
            sr2 = sigma_r * sigma_r
        tau = 2.0 * sr2 * NWIN * NWIN
        dl = ssd - ssd[:, 2:3]
        post = 1.0 / torch.exp(-dl / tau).sum(1)
        pi = omega[n] / wsum * post + pipar
        sig = None
        if n == f_lv and params["variance"]:
            xs = torch.tensor([o * o for o in OFFSETS], dtype=DT)
            ym = ssd.mean(1, keepdim=True)
            kappa = ((xs - xs.mean()) * (ssd - ym)).sum(1) / ((xs - xs.mean()) ** 2).sum()
            ok = (kappa > 0).detach()
            ks = torch.where(ok, kappa, torch.ones_like(kappa))
            res = (ssd - (ym + ks[:, None] * (xs - xs.mean()))) / tau
            mse = (res * res).mean(1)
            ok = ok & (mse <= params["var_fit_thresh"]).detach()
            s2 = tau / (2.0 * ks)
            ok_cap = ok & (s2 < sfail2).detach()
            sig = torch.where(ok_cap, s2, torch.full_like(s2, sfail2))
        # fusion (Eq. 9-13, 18) over accepted patches, scattered onto the level
        ka = torch.nonzero(acc).squeeze(1)
        pix = (Y[ka] * w + X[ka]).reshape(-1)
        Mk = M[None].expand(len(ka), P, P)
        W = Mk * pi[ka][:, None, None]
        z = torch.zeros(h * w, dtype=DT).index_add(0, pix, W.reshape(-1))
        zu = torch.zeros(h * w, dtype=DT).index_add(0, pix, (W * u[ka][:, None, None]).reshape(-1))
        zm = torch.zeros(h * w, dtype=DT).index_add(0, pix, Mk.reshape(-1))
        valid = (z > 0).detach()
        zs = torch.where(valid, z, torch.ones_like(z))
        zms = torch.where(valid, zm, torch.ones_like(zm))
        ub = zu / zs
        q = z / zms
        if n == f_lv:
            nanv = torch.full_like(ub, float("nan"))
            ok_px = valid
            if params["prob_thresh"] > 0:
                ok_px = ok_px & (q >= params["prob_thresh"]).detach()
            out["disp"] = torch.where(ok_px, -ub, nanv).reshape(h, w)
            out["conf"] = torch.where(ok_px, q, torch.zeros_like(q)).reshape(h, w)
            out["valid"] = ok_px.reshape(h, w)
            if sig is not None:
                zv = torch.zeros(h * w, dtype=DT).index_add(0, pix, (W * W * sig[ka][:, None, None]).reshape(-1))
                out["var"] = torch.where(ok_px, zv / (zs * zs), nanv).reshape(h, w)
        else:
            xs_ = torch.arange(w, dtype=DT)[None, :].expand(h, w).reshape(-1)
            ys_ = torch.arange(h, dtype=DT)[:, None].expand(h, w).reshape(-1)
            if par_u is not None:
                hu = 2.0 * _bilinear(par_u, 0.5 * xs_, 0.5 * ys_)
                hq = _bilinear(par_q, 0.5 * xs_, 0.5 * ys_)
            else:
                hu = torch.zeros(h * w, dtype=DT)
                hq = torch.zeros(h * w, dtype=DT)
            par_u = torch.where(valid, ub, hu).reshape(h, w)
            par_q = torch.where(valid, q, hq).reshape(h, w)
        trace.append(dict(level=n, u=u, acc=acc, ssd=ssd, post=post, pi=pi, tau=tau))
    out["levels"] = trace[::-1]
    return out


def hyper_tensors(params, requires_grad=True):
    """(sigma_s, sigma_r, omega) as float64 leaf tensors from a parameter dict."""
    ss = torch.tensor(float(params["sigma_s"]), dtype=DT, requires_grad=requires_grad)
    sr = torch.tensor(float(params["sigma_r"]), dtype=DT, requires_grad=requires_grad)
    om = torch.tensor([float(x) for x in params["level_weight"][:params["levels"]]], dtype=DT,
                      requires_grad=requires_grad)
    return ss, sr, om


def loss_and_grads(left, right, params, v_disp, v_var=None):
    """L = sum v_disp * disp + sum v_var * var over valid pixels, and its gradient
    with respect to (left, right, sigma_s, sigma_r, omega)."""
    lt = torch.tensor(left, dtype=DT, requires_grad=True)
    rt = torch.tensor(right, dtype=DT, requires_grad=True)
    ss, sr, om = hyper_tensors(params)
    out = forward(lt, rt, params, ss, sr, om)
    ok = out["valid"]
    loss = (torch.tensor(v_disp, dtype=DT)[ok] * out["disp"][ok]).sum()
    if v_var is not None:
        loss = loss + (torch.tensor(v_var, dtype=DT)[ok] * out["var"][ok]).sum()
    loss.backward()
    return dict(loss=float(loss.detach()), left=lt.grad.numpy(), right=rt.grad.numpy(), sigma_s=float(ss.grad),
                sigma_r=float(sr.grad), omega=om.grad.numpy(), out=out)

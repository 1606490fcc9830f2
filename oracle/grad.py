"""FP64 gradient oracle of the differentiable trace (Sec. 3.3, Stage II: the
trace is differentiable so gradients reach the surfels through the indirect
radiance).

TEST INFRASTRUCTURE (see the package docstring): never on the product path.

``grad_given_hits`` evaluates Eq. 6, 7 and the front-to-back blending of
Eq. 2 in float64 PyTorch over a *given* ordered hit list per ray and lets
autograd differentiate

    L = sum_r  g_O[r] O[r] + g_F[r] . F[r] + g_D[r] D[r]

with respect to the raw parameters (centre, raw quaternion, scales, opacity,
features).  Selection and order of the hits are piecewise constant in the
parameters, so they carry no gradient; the list is an input.

With ``sh_deg`` >= 0 the features are RGB coefficients of the real SH basis
and each hit contributes the colour max(Y(d).k + 1/2, 0) along the ray's
normalised direction d (3 output channels).  The basis here comes from
``scipy.special.sph_harm_y`` (an implementation independent of the C
oracle's recurrence).

``fd_grad`` takes central finite differences of the same L through the
brute-force C oracle (which re-selects and re-sorts the hits at each
perturbed point) and skips every parameter whose perturbation changes any
ray's ordered hit list.
"""
from __future__ import annotations

import numpy as np
import torch

from . import trace as _oracle_trace

_NAMES = ("mu", "quat", "scale", "opac", "feat")


def _frame(q):
    """t_u, t_v (first two rotation-matrix columns of the normalised
    quaternion (w,x,y,z)) and n = t_u x t_v."""
    qn = q / torch.linalg.vector_norm(q, dim=-1, keepdim=True)
    w, x, y, z = qn.unbind(-1)
    tu = torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y + w * z), 2 * (x * z - w * y)], -1)
    tv = torch.stack([2 * (x * y - w * z), 1 - 2 * (x * x + z * z), 2 * (y * z + w * x)], -1)
    n = torch.linalg.cross(tu, tv, dim=-1)
    return tu, tv, n


def sh_basis_scipy(rd, deg: int) -> np.ndarray:
    """Real SH basis Y[l*l + l + m] of the ray directions: sqrt(2) Re / sqrt(2)
    Im of scipy's complex harmonics (Condon-Shortley phase) for m > 0 / m < 0."""
    from scipy.special import sph_harm_y
    d = np.asarray(rd, np.float64).reshape(-1, 3)
    d = d / np.linalg.norm(d, axis=1, keepdims=True)
    polar = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    azim = np.arctan2(d[:, 1], d[:, 0])
    Y = np.zeros((d.shape[0], (deg + 1) ** 2))
    for l in range(deg + 1):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), polar, azim)
            Y[:, l * l + l + m] = c.real if m == 0 else np.sqrt(2.0) * (c.real if m > 0 else c.imag)
    return Y


def composite_given_hits(mu, quat, scale, opac, feat, ro, rd, lists, sh_deg: int = -1, with_normal: bool = False):
    """O, F, D, T of each ray from its ordered list (R, H) (-1 = padding).
    With ``with_normal`` (the relighting blend of albedo, roughness and
    normal with the same weights T alpha) F gains 3 channels: each hit's unit
    normal turned to face the ray, -n where n . d > 0; the turn is a
    piecewise-constant choice (no gradient), the normal itself carries the
    gradient to the raw quaternion."""
    valid = lists >= 0
    idx = lists.clamp(min=0)
    m = mu[idx]                                  # (R, H, 3)
    tu, tv, n = _frame(quat[idx])
    s = scale[idx]
    o = opac[idx]
    f = feat[idx]                                # (R, H, F)
    o_r = ro[:, None, :]
    d_r = rd[:, None, :]
    den = (n * d_r).sum(-1)
    den = torch.where(valid, den, torch.ones_like(den))
    tau = (n * (m - o_r)).sum(-1) / den          # Eq. 6
    p = o_r + tau[..., None] * d_r
    dlt = p - m
    u = (dlt * tu).sum(-1) / s[..., 0]           # Eq. 7
    v = (dlt * tv).sum(-1) / s[..., 1]
    alpha = o * torch.exp(-0.5 * (u * u + v * v))
    alpha = torch.where(valid, alpha, torch.zeros_like(alpha))
    tau = torch.where(valid, tau, torch.zeros_like(tau))
    one = torch.ones_like(alpha[:, :1])
    T = torch.cumprod(torch.cat([one, 1.0 - alpha[:, :-1]], 1), 1)   # Eq. 2
    w = T * alpha
    O = w.sum(1)
    if sh_deg >= 0:
        nb = (sh_deg + 1) ** 2
        Y = torch.tensor(sh_basis_scipy(rd.detach().numpy(), sh_deg))          # (R, nb), no gradient
        k = f.reshape(f.shape[0], f.shape[1], nb, 3)
        f = torch.relu((Y[:, None, :, None] * k).sum(2) + 0.5)                 # view-dependent colour
    if with_normal:
        sgn = torch.where((n * d_r).sum(-1) > 0, -1.0, 1.0).detach()
        f = torch.cat([f, sgn[..., None] * n], -1)
    F = (w[..., None] * f).sum(1)
    D = (w * tau).sum(1)
    Tend = T[:, -1] * (1.0 - alpha[:, -1]) if alpha.shape[1] else torch.ones_like(O)
    return O, F, D, Tend


def grad_given_hits(surfels, ro, rd, lists, gO, gF, gD, sh_deg: int = -1, with_normal: bool = False):
    """Gradients (dict of float64 numpy arrays) of L over given hit lists
    (with ``with_normal``, gF holds F + 3 channels: the features, then the
    facing normal)."""
    ts = [torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=True) for a in surfels]
    feat = ts[4].reshape(ts[0].shape[0], -1)
    ro_t = torch.tensor(np.asarray(ro, dtype=np.float64)).reshape(-1, 3)
    rd_t = torch.tensor(np.asarray(rd, dtype=np.float64)).reshape(-1, 3)
    L_t = torch.tensor(np.asarray(lists, dtype=np.int64))
    O, F, D, _ = composite_given_hits(ts[0], ts[1], ts[2], ts[3].reshape(-1), feat, ro_t, rd_t, L_t, sh_deg,
                                      with_normal)
    gO_t = torch.tensor(np.asarray(gO, dtype=np.float64)).reshape(-1)
    gF_t = torch.tensor(np.asarray(gF, dtype=np.float64)).reshape(O.shape[0], -1)
    gD_t = torch.tensor(np.asarray(gD, dtype=np.float64)).reshape(-1)
    L = (gO_t * O).sum() + (gF_t * F).sum() + (gD_t * D).sum()
    grads = torch.autograd.grad(L, ts, allow_unused=True)
    out = {}
    for name, t, g in zip(_NAMES, ts, grads):
        out[name] = np.zeros(t.shape) if g is None else g.detach().numpy()
    out["loss"] = float(L.detach())
    return out


def loss_and_hits(surfels, ro, rd, gO, gF, gD, hit_cap, **kw):
    r = _oracle_trace(surfels, ro, rd, hit_cap=hit_cap, **kw)
    L = float(np.sum(np.asarray(gO, np.float64) * r["O"]) +
              np.sum(np.asarray(gF, np.float64).reshape(r["F"].shape) * r["F"]) +
              np.sum(np.asarray(gD, np.float64) * r["D"]))
    return L, r


def fd_grad(surfels, ro, rd, gO, gF, gD, which=None, rel_h: float = 1e-6, hit_cap: int = 512,
            surfel_idx=None, **kw):
    """Central finite differences of L.  Returns (grads, skipped) where grads
    is a dict of arrays (NaN where skipped or not requested) and skipped
    counts the parameters whose +-h perturbation changed some ray's ordered
    hit list.  `surfel_idx` restricts the perturbed surfels."""
    base = [np.array(a, dtype=np.float64, copy=True) for a in surfels]
    _, ref = loss_and_hits(base, ro, rd, gO, gF, gD, hit_cap, **kw)
    ref_hits, ref_n = ref["hits"], ref["n_hits"]
    out = {}
    skipped = 0
    names = which or _NAMES
    for k, name in enumerate(_NAMES):
        if name not in names:
            continue
        arr = base[k]
        g = np.full(arr.shape, np.nan)
        flat = arr.reshape(-1)
        gflat = g.reshape(-1)
        per = flat.size // max(arr.shape[0], 1)
        rows = range(arr.shape[0]) if surfel_idx is None else surfel_idx
        for j in (int(r) * per + c for r in rows for c in range(per)):
            x0 = flat[j]
            h = rel_h * (abs(x0) if name == "scale" else max(1.0, abs(x0)))
            vals = []
            same = True
            for sgn in (1.0, -1.0):
                flat[j] = x0 + sgn * h
                Lp, rp = loss_and_hits(base, ro, rd, gO, gF, gD, hit_cap, **kw)
                if not (np.array_equal(rp["n_hits"], ref_n) and np.array_equal(rp["hits"], ref_hits)):
                    same = False
                vals.append(Lp)
            flat[j] = x0
            if same:
                gflat[j] = (vals[0] - vals[1]) / (2.0 * h)
            else:
                skipped += 1
        out[name] = g
    return out, skipped

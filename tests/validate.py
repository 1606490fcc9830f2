"""Per-ray acceptance of a GPU trace against the FP64 oracle.

A GPU list G of hit ids (in composite order) is accepted when:
  (i)   soundness   -- every id of G is an oracle hit or a threshold-ambiguous
                       near-hit;
  (ii)  order       -- consecutive FP64 depths of G never decrease by more than
                       the tie tolerance tol_ij;
  (iii) completeness-- every non-ambiguous oracle hit in front of G's last
                       depth (minus tol) is in G; if G did not terminate on the
                       cutoff, every non-ambiguous oracle hit is in G;
  (iv)  termination -- replaying G in FP64, T first drops below T_min exactly at
                       G's last hit (one-off allowed when T is within a band of
                       T_min);
then the GPU O, F, D, T must match the FP64 replay of G within `atol`.  Rays
with no tie and no ambiguous candidate must reproduce the oracle's own list
exactly.

Threshold ambiguity and tie tolerance scale with the FP32 error of the
kernel's depth: about 1e-6 (1 + |mu - r_o|) / |n . r_d| (the error of the
plane equation in FP32), turned into u, v error by the smallest scale.
"""
from __future__ import annotations

import numpy as np

import oracle

TIE_REL = 1e-6


def validate(surfels, ro, rd, gpu, rays=None, T_min=1e-4, alpha_min=1.0 / 255.0, sigma=3.0, t_min=0.0,
             t_max=np.inf, atol=1e-4, cap=4096, term_band=1e-4, sh_deg=-1, with_normal=False):
    """Returns a stats dict; raises AssertionError with a message on the
    first failing ray.  `gpu` holds numpy arrays O, F, D, T, n_hits, hit_ids."""
    ro = np.asarray(ro, np.float64)
    rd = np.asarray(rd, np.float64)
    R = ro.shape[0]
    rays = np.arange(R) if rays is None else np.asarray(rays)
    mu = np.asarray(surfels[0], np.float64)
    sc = np.asarray(surfels[2], np.float64)
    _, _, nrm = oracle.frames(surfels[1])
    sub_ro, sub_rd = ro[rays], rd[rays]
    cand = oracle.candidates(surfels, sub_ro, sub_rd, cap=cap, band=0.05, T_min=T_min, alpha_min=alpha_min,
                             sigma=sigma, t_min=t_min, t_max=t_max)
    ref = oracle.trace(surfels, sub_ro, sub_rd, hit_cap=cap, T_min=T_min, alpha_min=alpha_min, sigma=sigma, sh_deg=sh_deg, with_normal=with_normal,
                       t_min=t_min, t_max=t_max)
    H = gpu["hit_ids"].shape[1]
    nh = gpu["n_hits"][rays]
    assert np.all(nh <= H), "hit list capacity too small for validation"
    lists = np.ascontiguousarray(gpu["hit_ids"][rays])
    rep = oracle.replay(surfels, sub_ro, sub_rd, lists, nh, sh_deg=sh_deg, with_normal=with_normal)
    rep_ref = oracle.replay(surfels, sub_ro, sub_rd, ref["hits"], ref["n_hits"], sh_deg=sh_deg,
                            with_normal=with_normal)
    stats = dict(rays=len(rays), exact=0, exact_eligible=0, ambiguous_rays=0, tie_rays=0, hits=int(nh.sum()))
    for k, r in enumerate(rays):
        n = int(nh[k])
        G = lists[k, :n]
        cnt = int(cand["count"][k])
        assert cnt <= cap, f"ray {r}: more than {cap} candidates"
        ids = cand["ids"][k, :cnt]
        tau = cand["tau"][k, :cnt]
        rho2 = cand["rho2"][k, :cnt]
        alpha = cand["alpha"][k, :cnt]
        hit = cand["hit"][k, :cnt]
        cosn = np.abs(nrm[ids] @ rd[r]) / np.linalg.norm(rd[r])
        w = np.linalg.norm(mu[ids] - ro[r], axis=1)
        eps_tau = 4e-6 * (1.0 + w) / np.maximum(cosn, 1e-12)          # FP32 depth error bound
        eps_u = 2.0 * eps_tau / np.minimum(sc[ids, 0], sc[ids, 1])     # in units of the scale
        rho = np.sqrt(rho2)
        # with an infinite support radius (Eq. 5's proxy alone) only alpha_min decides the support
        sup_amb = (np.abs(rho2 - sigma * sigma) <= np.maximum(1e-3, 2 * sigma * eps_u)) if np.isfinite(sigma) \
            else np.zeros(cnt, bool)
        amb = (sup_amb |
               (np.abs(alpha - alpha_min) <= alpha_min * np.maximum(1e-3, rho * eps_u)) |
               (np.abs(tau - t_min) <= np.maximum(1e-6, eps_tau)) |
               (np.abs(tau - t_max) <= np.maximum(1e-6, eps_tau)))
        pos = {int(i): j for j, i in enumerate(ids)}
        ok_set = {int(i) for i, h, a in zip(ids, hit, amb) if h or a}
        # (i) soundness
        for g in G:
            assert int(g) in ok_set, f"ray {r}: GPU hit {g} is neither an oracle hit nor ambiguous"
        gt = np.array([tau[pos[int(g)]] for g in G])
        gc = np.array([cosn[pos[int(g)]] for g in G])
        # (ii) order
        for a in range(n - 1):
            tol = TIE_REL * max(1.0, abs(gt[a])) / min(gc[a], gc[a + 1]) + eps_tau[pos[int(G[a])]]
            assert gt[a + 1] >= gt[a] - tol, f"ray {r}: order violated at {a}: {gt[a]} > {gt[a+1]}"
        # (iv) termination
        Tp = rep["Tpost"][k, :n]
        terminated = n > 0 and Tp[-1] < T_min * (1 + term_band)
        if n > 1:
            early = np.nonzero(Tp[:-1] < T_min * (1 - term_band))[0]
            assert early.size == 0, f"ray {r}: FP64 replay crosses T_min at {early[0]} before the end {n-1}"
        if n > 0 and not terminated:
            assert Tp[-1] >= T_min * (1 - term_band), f"ray {r}: not terminated"
        # (iii) completeness
        Gs = set(int(g) for g in G)
        tlast = gt[-1] if n else -np.inf
        tol_last = TIE_REL * max(1.0, abs(tlast)) / max(gc.min() if n else 1.0, 1e-12) if n else 0.0
        for j in range(cnt):
            if hit[j] and not amb[j] and int(ids[j]) not in Gs:
                if terminated:
                    assert tau[j] >= tlast - tol_last - eps_tau[j], \
                        f"ray {r}: oracle hit {ids[j]} at tau {tau[j]} missing (last {tlast})"
                else:
                    raise AssertionError(f"ray {r}: oracle hit {ids[j]} missing from an unterminated list")
        # values against the FP64 replay of G
        for key, gv in (("O", gpu["O"][r]), ("D", gpu["D"][r]), ("T", gpu["T"][r])):
            assert abs(gv - rep[key][k]) <= atol, f"ray {r}: {key} {gv} vs replay {rep[key][k]}"
        assert np.all(np.abs(gpu["F"][r] - rep["F"][k]) <= atol), f"ray {r}: F differs from replay"
        # exactness where nothing is ambiguous and nothing ties
        any_amb = bool(np.any(amb))
        th = np.sort(tau[hit])
        ct = cosn[hit][np.argsort(tau[hit])] if hit.any() else np.zeros(0)
        ties = False
        if th.size > 1:
            tt = TIE_REL * np.maximum(1.0, np.abs(th[:-1])) / np.minimum(ct[:-1], ct[1:])
            ties = bool(np.any(np.diff(th) <= 2 * tt + 8e-6 * (1 + np.abs(th[:-1])) / np.minimum(ct[:-1], ct[1:])))
        nr = int(ref["n_hits"][k])
        near_cut = bool(np.any(np.abs(rep_ref["Tpost"][k, :nr] / T_min - 1.0) <= term_band)) if nr else False
        any_amb = any_amb or near_cut
        stats["ambiguous_rays"] += any_amb
        stats["tie_rays"] += ties
        if not any_amb and not ties:
            stats["exact_eligible"] += 1
            mine = ref["hits"][k, :ref["n_hits"][k]]
            assert n == ref["n_hits"][k] and np.array_equal(G, mine), \
                f"ray {r}: list differs from the oracle's on an unambiguous ray"
            stats["exact"] += 1
    return stats

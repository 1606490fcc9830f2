"""Helpers shared by the GPU tests: moving seeded inputs to the device and
results back.  No arithmetic of the method lives here."""
import sys

import numpy as np
import torch

DEV = torch.device("cuda:0") if torch.cuda.is_available() else None


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def make_scene(surfels, **kw):
    from paper_2412_15867_amd import Scene
    mu, q, s, o, f = (dev(x) for x in surfels.astuple()) if hasattr(surfels, "astuple") else (dev(x) for x in surfels)
    sc = Scene(mu, q, s, o, f, **kw)
    return sc


def to_np(res):
    out = {}
    for k, v in (("O", res.opacity), ("F", res.feat), ("D", res.depth), ("T", res.T), ("n_hits", res.n_hits),
                 ("hit_ids", res.hit_ids), ("hit_T", res.hit_T)):
        if v is not None:
            out[k] = v.detach().cpu().numpy()
    return out

"""Seeded synthetic systems drawn directly in device memory (large sizes).

Same recipe as ``synth.gen.gen`` (orbital energies sorted uniform in the
occupied and virtual ranges; per auxiliary index P a symmetric (Z + Z^T)/2 with
Z ~ N(0,1) scaled by 0.05/sqrt(naux), sliced into the oo/ov/vv blocks; three
dipole components 0.1 N(0,1) symmetrised, ov block kept), but drawn with
torch's Philox generator on the GPU, so the 200/800/3000 and 256/1024/4096
systems take seconds instead of minutes.  The random stream differs from the
numpy one; the distributions and shapes are the same.  Nothing here contracts,
divides or solves.
"""
from __future__ import annotations

import math


def gen_device(seed: int, o: int, v: int, naux: int, device: str = "cuda", chunk: int = 32):
    """Returns a dict of contiguous float64 device tensors: eps (o+v), B_oo (naux,o,o),
    B_ov (naux,o,v), B_vv (naux,v,v), dip (3,o,v)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    f64 = torch.float64
    e_o = torch.sort(torch.rand(o, generator=g, device=device, dtype=f64) * 0.7 - 1.0).values
    e_v = torch.sort(torch.rand(v, generator=g, device=device, dtype=f64) * 1.95 + 0.05).values
    n = o + v
    B_oo = torch.empty((naux, o, o), device=device, dtype=f64)
    B_ov = torch.empty((naux, o, v), device=device, dtype=f64)
    B_vv = torch.empty((naux, v, v), device=device, dtype=f64)
    pref = 0.05 / math.sqrt(naux)
    for p0 in range(0, naux, chunk):
        p1 = min(naux, p0 + chunk)
        Z = torch.randn((p1 - p0, n, n), generator=g, device=device, dtype=f64)
        S = (0.5 * pref) * (Z + Z.transpose(1, 2))
        B_oo[p0:p1] = S[:, :o, :o]
        B_ov[p0:p1] = S[:, :o, o:]
        B_vv[p0:p1] = S[:, o:, o:]
        del Z, S
    dip = torch.empty((3, o, v), device=device, dtype=f64)
    for x in range(3):
        Z = 0.1 * torch.randn((n, n), generator=g, device=device, dtype=f64)
        dip[x] = (0.5 * (Z + Z.T))[:o, o:]
    return dict(eps=torch.cat([e_o, e_v]).contiguous(), B_oo=B_oo, B_ov=B_ov, B_vv=B_vv, dip=dip.contiguous())

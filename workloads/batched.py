"""Batched-profile inputs: many independent profiles of very uneven size.

Profile sizes are lognormal(mu=13, sigma=1.5) samples clipped to [1e4, 2e7]
(natural-log parameters), drawn with numpy's Philox generator.  Each profile
uses one of a few program structures (function counts log-uniform in
[1e3, 5e4], 100 instructions and 10 source lines per function), has
max(32, functions / 10) placeholder contexts, and its records are drawn on the
GPU with torch's seeded generator: kernel-invocation segments of lognormal
length (mean 2,048) under a context drawn uniformly, a function by Zipf(1.1)
over a seeded hotness order, an instruction uniform within it, and a stall
reason from the instruction's Dirichlet(0.5) table.  This module only draws
inputs; it computes nothing of the attribution.
"""
from __future__ import annotations

import math

import numpy as np

from .gen import _build_structure, _rng, _stall_tables, STALL_TABLE, Workload, _C_ZIPF

_C_BATCH = 17


def batched_sizes(seed: int = 2109069313, n_profiles: int = 4096, mu: float = 13.0, sigma: float = 1.5,
                  lo: int = 10_000, hi: int = 20_000_000) -> np.ndarray:
    r = _rng(seed, _C_BATCH, 0)
    return np.clip(np.rint(r.lognormal(mu, sigma, size=n_profiles)), lo, hi).astype(np.int64)


def batched_structures(seed: int = 2109069313, n_struct: int = 4, lo: int = 1_000, hi: int = 50_000):
    """A few program structures with log-uniform function counts (the smallest
    and largest included); returns Workload objects (no samples) with the
    per-instruction data the sampler needs in .meta."""
    if n_struct == 1:
        counts = [lo]
    else:
        counts = [int(round(math.exp(math.log(lo) + (math.log(hi) - math.log(lo)) * k / (n_struct - 1))))
                  for k in range(n_struct)]
    out = []
    for k, v in enumerate(counts):
        rs = _rng(seed, _C_BATCH, 100 + k)
        sizes = np.full(v, 100, dtype=np.int64)
        st = _build_structure(rs, [(0x7000_0000_0000 + (k << 36), sizes)], 0, n_inline=v // 10, inline_depth=3,
                              n_loops=v // 10, n_lines=10 * v)
        w = Workload(name=f"batched-struct{k}", seed=seed, scope_start=st["scope_start"], scope_end=st["scope_end"],
                     scope_id=st["scope_id"], scope_kind=st["scope_kind"], line_start=st["line_start"],
                     line_end=st["line_end"], line_file=st["line_file"], line_line=st["line_line"],
                     n_scope_ids=st["n_scope_ids"], site_pc=np.zeros(0, np.uint64),
                     site_caller=np.zeros(0, np.uint32), site_callee=np.zeros(0, np.uint32),
                     ctx_parent=np.zeros(0, np.uint32), ctx_entry=np.zeros(0, np.int32), meta={"st": st})
        w.meta["n_funcs"] = st["n_funcs"]
        w.meta["n_ctx"] = max(32, st["n_funcs"] // 10)
        # Zipf(1.1) over a seeded hotness order of the functions
        rz = _rng(seed, _C_ZIPF, 200 + k)
        nf = st["n_funcs"]
        pw = np.arange(1, nf + 1, dtype=np.float64) ** -1.1
        cdf = np.cumsum(pw)
        cdf /= cdf[-1]
        w.meta["func_cdf"] = cdf
        w.meta["func_perm"] = rz.permutation(nf).astype(np.int64)
        w.meta["stall_tab"] = _stall_tables(_rng(seed, _C_BATCH, 300 + k), st["inst_pc"].shape[0])
        out.append(w)
    return out


class GpuSampler:
    """Draws a profile's records on the GPU (torch), for one structure."""

    def __init__(self, w: Workload, device="cuda"):
        import torch
        st = w.meta["st"]
        self.torch = torch
        self.n_ctx = w.meta["n_ctx"]
        self.cdf = torch.from_numpy(w.meta["func_cdf"]).to(device)
        self.perm = torch.from_numpy(w.meta["func_perm"]).to(device)
        self.optr = torch.from_numpy(st["owned_ptr"]).to(device)
        self.olist = torch.from_numpy(st["owned_list"]).to(device)
        self.inst_pc = torch.from_numpy(st["inst_pc"].view(np.int64)).to(device)
        self.tab = torch.from_numpy(w.meta["stall_tab"]).to(device)
        self.device = device

    def draw(self, seed: int, n: int, pc_out, ctx_out, stall_out):
        """Fill pc_out (int64 view), ctx_out (int32 view), stall_out (uint8) with n records."""
        torch = self.torch
        if n == 0:
            return
        rs = _rng(seed, _C_BATCH, 7)
        lens = []
        tot = 0
        mu = math.log(2048.0) - 0.5
        while tot < n:
            L = np.maximum(1, np.rint(rs.lognormal(mu, 1.0, size=max(16, 2 * n // 2048 + 16)))).astype(np.int64)
            lens.append(L)
            tot += int(L.sum())
        lens = np.concatenate(lens)
        cs = np.cumsum(lens)
        k = int(np.searchsorted(cs, n, side="left")) + 1
        lens = lens[:k].copy()
        lens[-1] -= int(cs[k - 1] - n)
        seg_ctx = rs.integers(0, self.n_ctx, size=k).astype(np.int32)
        ctx_out.copy_(torch.repeat_interleave(torch.from_numpy(seg_ctx).to(self.device),
                                              torch.from_numpy(lens).to(self.device)))
        g = torch.Generator(device=self.device)
        g.manual_seed(int(seed) & 0x7FFFFFFFFFFFFFFF)
        u = torch.rand(n, generator=g, device=self.device, dtype=torch.float64)
        f = self.perm[torch.clamp(torch.searchsorted(self.cdf, u), max=self.cdf.numel() - 1)]
        cnt = self.optr[f + 1] - self.optr[f]
        u2 = torch.rand(n, generator=g, device=self.device, dtype=torch.float64)
        off = torch.minimum((u2 * cnt).to(torch.int64), cnt - 1)
        inst = self.olist[self.optr[f] + off]
        pc_out.copy_(self.inst_pc[inst])
        u3 = torch.rand(n, generator=g, device=self.device)
        col = torch.clamp((u3 * STALL_TABLE).to(torch.int64), max=STALL_TABLE - 1)
        stall_out.copy_(self.tab[inst, col])

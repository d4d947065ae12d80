"""Plain reference of cross-profile unification, statistics and the sparse
formats -- test infrastructure only.

Inputs are several profiles' attributions over one structure map and context
table: per profile, keys (ctx, pc, stall) with integer counts.

- Unification (Section 6.1, call path profile unification): the union of the
  profiles' (ctx, pc) contexts, sorted, numbered 0..U-1.
- Metrics: metric m is the sample count with stall reason m (m = 0..15).
- Statistics (Section 4.5 derived metrics combining profiles): for every
  (context, metric) with a non-zero value in some profile, over all P
  profiles, a profile without the key counting as 0: sum, min, max, mean =
  sum / P, population standard deviation sqrt(sum_p (x_p - mean)^2 / P) and
  coefficient of variation std / mean.
- CMS (Section 6.2, CCT-major sparse): per context, its non-empty metrics as
  (metric, start) pairs into pids / vals, entries ordered by metric then
  profile.  PMS (profile-major sparse): per profile, its (context, metric,
  value) triples ordered by context then metric, with (context, start) pairs
  for the contexts it has.

Plain Python dictionaries and loops; nothing is shared with the library.
"""
from __future__ import annotations

import math

import numpy as np

NS = 16


def _keys(a):
    """Dict (ctx, pc, stall) -> count of one attribution-like object."""
    return {(int(c), int(p), int(s)): int(n) for c, p, s, n in zip(a.ctx, a.pc, a.stall, a.count)}


def unify(profiles):
    """profiles: attribution-like objects (ctx, pc, stall, count arrays).
    Returns a dict with the unified contexts, CMS, PMS and statistics."""
    P = len(profiles)
    keys = [_keys(a) for a in profiles]
    ctxs = sorted({(c, p) for k in keys for (c, p, _) in k})
    cid = {cp: i for i, cp in enumerate(ctxs)}
    # CMS
    cms_ctx_off = [0]
    cms_m_off = [0]
    cms_mid, cms_mstart, cms_pid, cms_val = [], [], [], []
    stats = []
    for (c, p) in ctxs:
        for m in range(NS):
            vals = [(q, keys[q].get((c, p, m), 0)) for q in range(P)]
            nz = [(q, v) for q, v in vals if v > 0]
            if not nz:
                continue
            cms_mid.append(m)
            cms_mstart.append(len(cms_pid))
            for q, v in nz:
                cms_pid.append(q)
                cms_val.append(v)
            xs = [v for _, v in vals]
            s = sum(xs)
            mean = s / P
            var = sum((x - mean) ** 2 for x in xs) / P
            std = math.sqrt(var)
            stats.append((cid[(c, p)], m, s, min(xs), max(xs), mean, std, std / mean if mean > 0 else 0.0))
        cms_ctx_off.append(len(cms_pid))
        cms_m_off.append(len(cms_mid))
    # PMS
    pms_off, pms_c_off = [0], [0]
    pms_ctx, pms_cstart, pms_mid, pms_val = [], [], [], []
    for q in range(P):
        last = None
        for (c, p, m) in sorted(keys[q]):
            u = cid[(c, p)]
            if u != last:
                pms_ctx.append(u)
                pms_cstart.append(len(pms_mid))
                last = u
            pms_mid.append(m)
            pms_val.append(keys[q][(c, p, m)])
        pms_off.append(len(pms_mid))
        pms_c_off.append(len(pms_ctx))
    st = np.array([s[:5] for s in stats], dtype=np.uint64).reshape(-1, 5)
    fl = np.array([s[5:] for s in stats], dtype=np.float64).reshape(-1, 3)
    return dict(
        ctx=np.array([c for c, _ in ctxs], np.uint32), pc=np.array([p for _, p in ctxs], np.uint64),
        cms_ctx_off=np.array(cms_ctx_off, np.uint64), cms_m_off=np.array(cms_m_off, np.uint64),
        cms_mid=np.array(cms_mid, np.uint8), cms_mstart=np.array(cms_mstart, np.uint64),
        cms_pid=np.array(cms_pid, np.uint32), cms_val=np.array(cms_val, np.uint64),
        pms_off=np.array(pms_off, np.uint64), pms_c_off=np.array(pms_c_off, np.uint64),
        pms_ctx=np.array(pms_ctx, np.uint32), pms_cstart=np.array(pms_cstart, np.uint64),
        pms_mid=np.array(pms_mid, np.uint8), pms_val=np.array(pms_val, np.uint64),
        st_ctx=st[:, 0].astype(np.uint32), st_mid=st[:, 1].astype(np.uint8), st_sum=st[:, 2], st_min=st[:, 3],
        st_max=st[:, 4], st_mean=fl[:, 0], st_std=fl[:, 1], st_cov=fl[:, 2])


def combine(profiles):
    """Multi-run combination (Section 4.7): per key, the sum of the runs' counts,
    keys sorted by (ctx, pc, stall)."""
    tot = {}
    for a in profiles:
        for k, v in _keys(a).items():
            tot[k] = tot.get(k, 0) + v
    ks = sorted(tot)
    return dict(ctx=np.array([k[0] for k in ks], np.uint32), pc=np.array([k[1] for k in ks], np.uint64),
                stall=np.array([k[2] for k in ks], np.uint8), count=np.array([tot[k] for k in ks], np.uint64))

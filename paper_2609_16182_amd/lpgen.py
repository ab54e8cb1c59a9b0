"""Seeded synthetic LP generators.

This module only draws random problem data. It holds none of the presolve
arithmetic, so both the CPU oracle and the GPU path can be fed from it.

Every generator returns a dict with the LP in the form of eq. (1) of the paper
(section 2.1): minimize c'x s.t. lhs <= Ax <= rhs, lb <= x <= ub, with A in CSR
(int32 row_ptr / col_idx, float64 val, column indices ascending in each row),
plus the feasible point ``x0`` the sides were built from and the index lists of
the planted reductions.

Value, bound and side recipe (shared by all workloads):
  * coefficients +-U[0.5, 2], 10% of them set to +-1 (uniform sign);
  * rows: 40% equality, 40% one-sided <=, 20% ranged; sides from x0:
    equality lhs = rhs = a.x0; <= rhs = a.x0 + U[0,1]; ranged a.x0 -+ U[0,1];
  * bounds: 40% [0, inf), 40% [0, U[1,10]], 20% free;
    x0_j ~ U[0, min(5, ub_j)] (free columns U[0, 5]);
  * costs: boxed columns U[-1,1], [0,inf) columns U[0,1], free columns 0, and
    10% of all costs zeroed, so every LP is bounded below.
"""
from __future__ import annotations

import numpy as np

INF = np.inf

ROW_EQ, ROW_LE, ROW_RANGED = 0, 1, 2


def _values(rng, k):
    mag = rng.uniform(0.5, 2.0, size=k)
    unit = rng.random(k) < 0.10
    mag[unit] = 1.0
    sign = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    return sign * mag


def _bounds(rng, n):
    kind = rng.choice(3, size=n, p=[0.4, 0.4, 0.2])  # 0: [0,inf) 1: [0,U] 2: free
    lb = np.zeros(n)
    ub = np.full(n, INF)
    boxed = kind == 1
    ub[boxed] = rng.uniform(1.0, 10.0, size=int(boxed.sum()))
    free = kind == 2
    lb[free] = -INF
    x0 = rng.uniform(0.0, 1.0, size=n) * np.minimum(5.0, ub)
    c = np.zeros(n)
    c[boxed] = rng.uniform(-1.0, 1.0, size=int(boxed.sum()))
    half = kind == 0
    c[half] = rng.uniform(0.0, 1.0, size=int(half.sum()))
    c[rng.random(n) < 0.10] = 0.0
    return lb, ub, x0, c, kind


def _uniform_cols(n):
    def draw(rng, k):
        return rng.integers(0, n, size=k, dtype=np.int64)
    return draw


def _powerlaw_cols(rng, n, exponent=1.0):
    """Column choice proportional to (rank+1)^-exponent over a seeded permutation."""
    perm = rng.permutation(n).astype(np.int64)
    w = 1.0 / np.power(np.arange(1, n + 1, dtype=np.float64), exponent)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]

    def draw(rng2, k):
        r = np.searchsorted(cdf, rng2.random(k), side="right")
        np.minimum(r, n - 1, out=r)
        return perm[r]
    return draw


def _fill_columns(rng, lengths, n, draw):
    """Distinct, ascending column indices for every row (sampling without
    replacement by redrawing duplicates)."""
    m = len(lengths)
    row_of = np.repeat(np.arange(m, dtype=np.int64), lengths)
    cols = draw(rng, len(row_of))
    key = row_of * n + cols
    key.sort()
    for it in range(10_000):
        dup = np.flatnonzero(key[1:] == key[:-1]) + 1
        if len(dup) == 0:
            break
        # after many redraws from a skewed law, finish with uniform redraws
        new = draw(rng, len(dup)) if it < 48 else rng.integers(0, n, size=len(dup))
        key[dup] = row_of[dup] * n + new
        key.sort()
    return (key % n).astype(np.int32)


def _row_ptr(lengths):
    rp = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=rp[1:])
    return rp


def _sides(rng, act, kinds):
    m = len(act)
    lhs = np.empty(m)
    rhs = np.empty(m)
    eq = kinds == ROW_EQ
    le = kinds == ROW_LE
    rg = kinds == ROW_RANGED
    lhs[eq] = act[eq]
    rhs[eq] = act[eq]
    lhs[le] = -INF
    rhs[le] = act[le] + rng.uniform(0.0, 1.0, size=int(le.sum()))
    lhs[rg] = act[rg] - rng.uniform(0.0, 1.0, size=int(rg.sum()))
    rhs[rg] = act[rg] + rng.uniform(0.0, 1.0, size=int(rg.sum()))
    return lhs, rhs


def _activity_at(row_ptr, col_idx, val, x0):
    m = len(row_ptr) - 1
    rows = np.repeat(np.arange(m), np.diff(row_ptr))
    return np.bincount(rows, weights=val * x0[col_idx], minlength=m)


def make_lp(m, n, *, seed, row_len=(4, 8), col_dist="uniform", zipf_cap=None,
            singleton=0, empty=0, doubleton=0, duplicate=0, fixed_cols=0,
            dense_rows=(0, 0), dense_cols=(0, 0), chains=0, chain_len=8):
    """General synthetic LP.

    row_len: (lo, hi) for U{lo..hi}, or ("zipf", s) for 2 + Zipf(s) capped at
    ``zipf_cap``.  Planted counts are numbers of rows (columns for fixed_cols).
    dense_rows = (count, length); dense_cols = (count, rows each).
    chains = number of planted propagation chains of ``chain_len`` rows, each
    moving a finite upper bound one row further per Jacobi round.
    """
    rng = np.random.default_rng(seed)
    lb, ub, x0, c, bkind = _bounds(rng, n)

    # --- reserve columns for chains (kept out of the random rows) ---------
    n_chain_cols = chains * (chain_len + 1 + 2 * chain_len)
    if n_chain_cols > n // 4:
        raise ValueError("too many chains for n")
    chain_cols = np.arange(n - n_chain_cols, n, dtype=np.int64)
    n_rand = n - n_chain_cols

    # --- row lengths -------------------------------------------------------
    n_plain = m - chains * chain_len
    if isinstance(row_len, tuple) and len(row_len) == 2 and row_len[0] == "zipf":
        z = rng.zipf(row_len[1], size=n_plain).astype(np.int64)
        lengths = 2 + z
        cap = zipf_cap if zipf_cap is not None else n_rand
        np.minimum(lengths, min(cap, max(2, n_rand // 4)), out=lengths)
    else:
        lengths = rng.integers(row_len[0], row_len[1] + 1, size=n_plain).astype(np.int64)

    planted_total = singleton + empty + doubleton + duplicate + dense_rows[0]
    if planted_total > n_plain:
        raise ValueError("too many planted rows")
    perm = rng.permutation(n_plain)
    o = 0
    sing_rows = np.sort(perm[o:o + singleton]); o += singleton
    empty_rows = np.sort(perm[o:o + empty]); o += empty
    dbl_rows = np.sort(perm[o:o + doubleton]); o += doubleton
    dup_rows = perm[o:o + duplicate]; o += duplicate
    dense_row_ids = np.sort(perm[o:o + dense_rows[0]]); o += dense_rows[0]
    normal_rows = perm[o:]
    dup_src = rng.choice(normal_rows, size=duplicate, replace=True) if duplicate else np.zeros(0, np.int64)

    lengths[sing_rows] = 1
    lengths[empty_rows] = 0
    lengths[dbl_rows] = 2
    lengths[dup_rows] = lengths[dup_src]
    if dense_rows[0]:
        lengths[dense_row_ids] = min(dense_rows[1], n_rand)

    draw = _uniform_cols(n_rand) if col_dist == "uniform" else _powerlaw_cols(rng, n_rand)
    cols = _fill_columns(rng, lengths, n_rand, draw)
    rp = _row_ptr(lengths)
    vals = _values(rng, len(cols))

    # duplicates copy their source's pattern with coefficients scaled by lambda
    lam = np.zeros(duplicate)
    if duplicate:
        lam = rng.uniform(0.5, 3.0, size=duplicate) * np.where(rng.random(duplicate) < 0.5, -1.0, 1.0)
        for d, s, l in zip(dup_rows, dup_src, lam):
            cols[rp[d]:rp[d + 1]] = cols[rp[s]:rp[s + 1]]
            vals[rp[d]:rp[d + 1]] = vals[rp[s]:rp[s + 1]] * l

    # --- dense columns: inserted into random rows (existing entries kept) --
    if dense_cols[0]:
        dcols = rng.choice(n_rand, size=dense_cols[0], replace=False)
        nrows = min(dense_cols[1], n_plain)
        extra_r = np.concatenate([rng.choice(n_plain, size=nrows, replace=False) for _ in dcols])
        extra_c = np.repeat(dcols.astype(np.int64), nrows)
        row_of = np.repeat(np.arange(n_plain, dtype=np.int64), lengths)
        key_old = row_of * n_rand + cols
        key_new = extra_r * n_rand + extra_c
        keep_new = ~np.isin(key_new, key_old)
        # the planted rows (singleton/empty/doubleton/duplicate) keep their shape
        special = np.zeros(n_plain, bool)
        special[sing_rows] = special[empty_rows] = special[dbl_rows] = True
        special[dup_rows] = special[dup_src] = True
        keep_new &= ~special[extra_r]
        key_all = np.concatenate([key_old, key_new[keep_new]])
        val_all = np.concatenate([vals, _values(rng, int(keep_new.sum()))])
        order = np.argsort(key_all, kind="stable")
        key_all = key_all[order]
        vals = val_all[order]
        cols = (key_all % n_rand).astype(np.int32)
        lengths = np.bincount((key_all // n_rand).astype(np.int64), minlength=n_plain)
        rp = _row_ptr(lengths)

    # --- fixed columns: lb = ub = x0 ---------------------------------------
    fixed = np.zeros(0, np.int64)
    if fixed_cols:
        fixed = np.sort(rng.choice(n_rand, size=fixed_cols, replace=False))
        lb[fixed] = x0[fixed]
        ub[fixed] = x0[fixed]
        c[fixed] = rng.uniform(-1.0, 1.0, size=fixed_cols)

    # --- row kinds and sides -------------------------------------------------
    kinds = rng.choice(3, size=n_plain, p=[0.4, 0.4, 0.2])
    kinds[dbl_rows] = ROW_EQ
    act = _activity_at(rp, cols, vals, x0[:n_rand])
    lhs, rhs = _sides(rng, act, kinds)
    er_kind = rng.random(len(empty_rows)) < 0.5
    lhs[empty_rows] = np.where(er_kind, -INF, -rng.uniform(0, 1, len(empty_rows)))
    rhs[empty_rows] = rng.uniform(0, 1, len(empty_rows))
    if duplicate:
        sl, sr = lhs[dup_src], rhs[dup_src]
        lhs[dup_rows] = np.where(lam > 0, sl * lam, sr * lam)
        rhs[dup_rows] = np.where(lam > 0, sr * lam, sl * lam)

    # --- planted propagation chains: y_{k+1} - y_k + sum a_e x_e <= 0 -------
    ch_rp_parts, ch_cols, ch_vals, ch_lhs, ch_rhs = [], [], [], [], []
    for t in range(chains):
        base = chain_cols[t * (3 * chain_len + 1)]
        ys = base + np.arange(chain_len + 1)
        xs = base + chain_len + 1 + np.arange(2 * chain_len)
        lb[ys] = 0.0
        ub[ys] = INF
        ub[ys[0]] = 1.0
        x0[ys] = 0.0
        lb[xs] = 0.0
        ub[xs] = rng.uniform(1.0, 10.0, size=len(xs))
        x0[xs] = 0.0
        c[ys] = 0.0
        c[xs] = rng.uniform(0.0, 1.0, size=len(xs))
        for k in range(chain_len):
            row = sorted([(int(ys[k]), -1.0), (int(ys[k + 1]), 1.0),
                          (int(xs[2 * k]), float(rng.uniform(0.5, 2.0))),
                          (int(xs[2 * k + 1]), float(rng.uniform(0.5, 2.0)))])
            ch_rp_parts.append(len(row))
            ch_cols.extend(r[0] for r in row)
            ch_vals.extend(r[1] for r in row)
            ch_lhs.append(-INF)
            ch_rhs.append(0.0)
    if chains:
        lengths = np.concatenate([np.diff(rp), np.array(ch_rp_parts, np.int64)])
        rp = _row_ptr(lengths)
        cols = np.concatenate([cols, np.array(ch_cols, np.int32)])
        vals = np.concatenate([vals, np.array(ch_vals)])
        lhs = np.concatenate([lhs, np.array(ch_lhs)])
        rhs = np.concatenate([rhs, np.array(ch_rhs)])

    if rp[-1] >= 2 ** 31:
        raise ValueError("nnz exceeds int32 indexing")
    return {
        "m": int(m), "n": int(n),
        "row_ptr": rp.astype(np.int32), "col_idx": np.ascontiguousarray(cols, np.int32),
        "val": np.ascontiguousarray(vals, np.float64),
        "lhs": lhs, "rhs": rhs, "lb": lb, "ub": ub, "c": c, "obj_offset": 0.0,
        "x0": x0,
        "planted": {
            "singleton_rows": sing_rows, "empty_rows": empty_rows,
            "doubleton_rows": dbl_rows, "duplicate_rows": np.sort(dup_rows),
            "duplicate_pairs": np.stack([dup_rows, dup_src]).astype(np.int64),
            "fixed_cols": fixed,
            "dense_rows": dense_row_ids, "chain_rows": np.arange(n_plain, m),
        },
    }


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

def single_small(seed=0):
    """Single synthetic LP: m=2000, n=3000, U{4..8} nnz/row, uniform columns,
    planted 50 singleton, 50 empty, 100 doubleton-equality, 50 duplicate rows
    and 100 lb=ub columns."""
    return make_lp(2000, 3000, seed=seed, row_len=(4, 8), singleton=50, empty=50,
                   doubleton=100, duplicate=50, fixed_cols=100)


def power_law(seed=1, scale=1.0):
    """Power-law LP: m=1e6*scale, n=1.5m, row length 2+Zipf(2) capped at 1e5,
    power-law (exponent 1) column choice; 2% of rows planted (1/3 singleton,
    1/3 doubleton, 1/3 scaled duplicates)."""
    m = max(200, int(round(1_000_000 * scale)))
    n = int(round(1.5 * m))
    k = int(0.02 * m) // 3
    return make_lp(m, n, seed=seed, row_len=("zipf", 2.0), zipf_cap=100_000,
                   col_dist="powerlaw", singleton=k, doubleton=k, duplicate=k)


def large(seed=2, scale=1.0):
    """Large LP: m=1e7*scale, n=1.5m, U{3..12} nnz/row, uniform columns, 20
    dense rows of 1e6*scale entries, 20 dense columns in 1e5*scale rows each,
    1% planted rows including 8-row propagation chains."""
    m = max(2000, int(round(10_000_000 * scale)))
    n = int(round(1.5 * m))
    k = int(0.01 * m)
    chains = max(1, k // 40)
    rest = k - chains * 8
    d_len = max(1000, int(round(1_000_000 * scale)))
    d_rows = max(100, int(round(100_000 * scale)))
    return make_lp(m, n, seed=seed, row_len=(3, 12), singleton=rest // 3,
                   doubleton=rest // 3, duplicate=rest - 2 * (rest // 3),
                   dense_rows=(20, d_len), dense_cols=(20, d_rows), chains=chains)


def batch_member(index, m=None, seed_base=3):
    """One LP of the batched workload: m log-uniform in [100, 20000],
    n = 1.5m, U{4..10} nnz/row, planted in the same ratios as the small LP."""
    rng = np.random.default_rng(seed_base + index)
    if m is None:
        m = int(round(np.exp(rng.uniform(np.log(100), np.log(20000)))))
    n = int(round(1.5 * m))
    f = m / 2000.0
    return make_lp(m, n, seed=seed_base + index + 7919, row_len=(4, 10),
                   singleton=int(50 * f), empty=int(50 * f), doubleton=int(100 * f),
                   duplicate=int(50 * f), fixed_cols=int(100 * f))


def serving_member(index, m_lo=1_000, m_hi=1_000_000, seed_base=4):
    """One LP of the serving pool: m log-uniform in [m_lo, m_hi], n = 1.5m,
    U{4..20} nnz/row, small-LP planting ratios."""
    rng = np.random.default_rng(seed_base + index)
    m = int(round(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi)))))
    n = int(round(1.5 * m))
    f = m / 2000.0
    return make_lp(m, n, seed=seed_base + index + 104729, row_len=(4, 20),
                   singleton=int(50 * f), empty=int(50 * f), doubleton=int(100 * f),
                   duplicate=int(50 * f), fixed_cols=int(100 * f))


def tiny(seed, m=None, n=None, finite_bounds=False):
    """Tiny LP (m, n <= 6) for brute-force checks; mixes every row and bound
    kind and sometimes plants a duplicate row, a singleton row, an empty row or
    a fixed column."""
    rng = np.random.default_rng(10_000 + seed)
    if m is None:
        m = int(rng.integers(1, 6))
    if n is None:
        n = int(rng.integers(1, 5))
    lb = np.zeros(n)
    ub = np.zeros(n)
    for j in range(n):
        k = rng.integers(0, 4 if not finite_bounds else 2)
        if k == 0:
            lb[j], ub[j] = 0.0, float(rng.integers(1, 6))
        elif k == 1:
            lb[j], ub[j] = float(-rng.integers(0, 3)), float(rng.integers(1, 4))
        elif k == 2:
            lb[j], ub[j] = 0.0, INF
        else:
            lb[j], ub[j] = -INF, INF
    u = rng.random(n)
    with np.errstate(invalid="ignore"):
        x0 = np.where(np.isfinite(ub), lb + (np.minimum(ub, lb + 5) - lb) * u,
                      np.where(np.isfinite(lb), lb, 0.0) + 3 * rng.random(n))
    x0 = np.round(x0 * 4) / 4
    rows = []
    for i in range(m):
        L = int(rng.integers(0, n + 1))
        cols = np.sort(rng.choice(n, size=L, replace=False)) if L else np.zeros(0, int)
        vals = rng.choice([-2.0, -1.5, -1.0, -0.5, 0.5, 1.0, 2.0, 3.0], size=L)
        rows.append([cols, vals])
    if m >= 2 and rng.random() < 0.4:
        src = int(rng.integers(0, m))
        dst = int(rng.integers(0, m))
        if src != dst and len(rows[src][0]) >= 2:
            lam = float(rng.choice([-2.0, -0.5, 0.5, 2.0, 3.0]))
            rows[dst] = [rows[src][0].copy(), rows[src][1] * lam]
    if n >= 1 and rng.random() < 0.3:
        j = int(rng.integers(0, n))
        if np.isfinite(lb[j]) and np.isfinite(ub[j]):
            lb[j] = ub[j] = x0[j]
    row_ptr = np.zeros(m + 1, np.int64)
    for i, (cc, _) in enumerate(rows):
        row_ptr[i + 1] = row_ptr[i] + len(cc)
    col_idx = np.concatenate([r[0] for r in rows]).astype(np.int32) if row_ptr[-1] else np.zeros(0, np.int32)
    val = np.concatenate([r[1] for r in rows]).astype(np.float64) if row_ptr[-1] else np.zeros(0)
    act = _activity_at(row_ptr, col_idx, val, x0)
    kinds = rng.choice(3, size=m, p=[0.3, 0.4, 0.3])
    lhs = np.empty(m)
    rhs = np.empty(m)
    for i in range(m):
        slack = float(rng.choice([0.0, 0.5, 1.0, 2.0]))
        if kinds[i] == ROW_EQ:
            lhs[i] = rhs[i] = act[i]
        elif kinds[i] == ROW_LE:
            lhs[i], rhs[i] = -INF, act[i] + slack
        else:
            lhs[i], rhs[i] = act[i] - slack, act[i] + float(rng.choice([0.0, 1.0, 3.0]))
        if rng.random() < 0.1:
            lhs[i], rhs[i] = -INF, INF
    c = rng.choice([-2.0, -1.0, 0.0, 1.0, 2.0], size=n)
    return {
        "m": m, "n": n, "row_ptr": row_ptr.astype(np.int32), "col_idx": col_idx,
        "val": val, "lhs": lhs, "rhs": rhs, "lb": lb, "ub": ub, "c": c,
        "obj_offset": 0.0, "x0": x0, "planted": {},
    }


def nnz(lp):
    return int(lp["row_ptr"][-1])

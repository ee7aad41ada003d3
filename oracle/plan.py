"""Independent implementation of the written integer plan rules (test infrastructure).

The HIP library's planner must produce exactly these integers.  Rules:

P1  Effective order: De = largest d with R_d > 0 (De = 2 if every rank is 0).
P2  FFT length: L = max(16, smallest power of two >= De*N - 1).  A cyclic
    length L keeps every gain output k in [2, N] free of wrap-around for every
    d <= De, because k + L > d*N for k >= 2.  M = L/2 is the complex length of
    the half-length transform that carries a real length-L transform.
P3  Column ids: scan d = 2..D ascending, m = 1..d, r = 1..R_d; the column
    U^(d)_m(:, r) gets the id of the first earlier column that is bitwise equal
    (all N binary64 words), else the next new id.  u = number of ids.  Without
    sharing (the plain reference evaluation) every column gets a new id.
P4  Gain terms: for each (d, r) the key is the ascending-sorted tuple of the d
    column ids; equal keys merge and count a multiplicity.  Order: by d, then
    lexicographic key.  Coefficient = multiplicity / d!.
P5  Loss terms: for each (d, r) the key is (d, id of mode d, ascending-sorted ids
    of modes 1..d-1); equal keys merge with multiplicity.  Order: by that key.
    Coefficient = multiplicity / (d-1)!.
P6  Two-pass split: lg = log2 M; M1 = 2^ceil(lg/2), M2 = M/M1.  With cs = 16
    bytes per stored complex (fp64, fp32c) or 8 (fp32): while u*2*M2*cs > 64 KiB
    and M1 < 2048, double M1 and halve M2.  Unsupported if then M1 > 2048 or
    M2 < 2 (more than 1024 distinct columns at the shortest lengths).
P7  Column tile: g = min(M2, max(1, 1024 / M1)) adjacent columns per workgroup.
P8  Row-pass chunks, only when u*2*(M2 + M2/16)*cs + (M2 <= 512 ? M2*cs : 0)
    > 144 KiB after P6 (the combine cannot hold every column's two padded rows
    and the row twiddles at once): cmax = floor(148 KiB / (2*(M2 +
    M2/16)*cs)) columns per chunk (rows padded by one slot in 16 in LDS).  Gain terms are visited in the order of their ascending
    tuple of distinct ids, ties kept in P4 order; a chunk takes the next term
    while the union of its distinct ids and the term's stays within cmax, else
    the chunk closes and a new one starts with that term.  Unsupported if a
    single term has more than cmax distinct ids.  A chunk lists its ids
    ascending and its terms by P4 position, in visiting order.

With the mixed-radix option (transform lengths 3 2^a and 5 2^a):

X2  L' = the smaller of the smallest 48*2^k and the smallest 80*2^k (k >= 0)
    that are >= De*N - 1.  Only when L' < L (P2) is it tried; else P2/P6/P7.
X6  With M = L'/2 = o 2^m (o = 3 or 5): M2 = largest power of two with M2^2
    <= M, M1 = M/M2.  While M1 > M1max (1536 for o = 3, 1280 for o = 5) and
    2*o divides M1: halve M1, double M2.  Then while u*2*M2*cs > 64 KiB,
    2*M1 <= M1max and M2 >= 4: double M1, halve M2.  The split is kept when
    M1 lies in [M1min, M1max] (M1min 96 for o = 3, 160 for o = 5), o divides
    M1, M2 >= 2, and 2^b divides L' with b = ceil(ceil(log2 L')/2) (the
    two-level table of w_L' splits the exponent at bit b); otherwise L, P6
    and P7 are used as without the option.
X7  g = the largest power of two <= min(M2, max(1, floor(1024 / M1))).
P8 applies unchanged with the M2 of X6.

Flat table (int64), as exported for comparison:
    [L, M1, M2, g, u, Tp, Tq, De,
     colmap in scan order (one id per (d, m, r)),
     per gain term:  d, multiplicity, ids[d],
     per loss term:  d, multiplicity, kmode id, ids[d-1],
     nchunks (0 without P8), per chunk: ncols, nterms, ids[ncols], terms[nterms]]
"""
from __future__ import annotations

import numpy as np

PREC_BYTES = {"fp64": 16, "fp32": 8, "fp32c": 16}


class Unsupported(ValueError):
    pass


def _log2_exact(x: int) -> int:
    assert x > 0 and (x & (x - 1)) == 0
    return x.bit_length() - 1


def _ceil_log2(x: int) -> int:
    return (x - 1).bit_length()


def _mixed_split(L: int, u: int, cs: int):
    """X6/X7 for a length L' = o 2^a: (M1, M2, g), or None when unsupported."""
    o = 3 if L % 3 == 0 else 5
    M = L // 2
    M1max, M1min = (1536, 96) if o == 3 else (1280, 160)
    M2 = 1
    while (2 * M2) ** 2 <= M:
        M2 *= 2
    M1 = M // M2
    while M1 > M1max and M1 % (2 * o) == 0:
        M1 //= 2
        M2 *= 2
    while u * 2 * M2 * cs > 65536 and 2 * M1 <= M1max and M2 >= 4:
        M1 *= 2
        M2 //= 2
    b = (_ceil_log2(L) + 1) // 2
    if not (M1min <= M1 <= M1max and M1 % o == 0 and M2 >= 2 and L % (1 << b) == 0):
        return None
    cap = min(M2, max(1, 1024 // M1))
    g = 1
    while 2 * g <= cap:
        g *= 2
    return M1, M2, g


def plan_tables(D: int, N: int, kernel: dict, prec: str = "fp64", dedup: bool = True, mixed: bool = False):
    ranks = {d: (kernel[d].shape[1] if d in kernel else 0) for d in range(2, D + 1)}
    De = max([d for d in range(2, D + 1) if ranks[d] > 0], default=2)
    L = 1
    while L < De * N - 1:
        L *= 2
    L = max(16, L)
    M = L // 2

    ids = []          # list of bytes for each distinct column
    colmap = []
    cmap = {}
    for d in range(2, D + 1):
        for m in range(d):
            for r in range(ranks[d]):
                key = np.ascontiguousarray(kernel[d][m, r], dtype=np.float64).tobytes()
                found = -1
                for j, kk in enumerate(ids):
                    if dedup and kk == key:
                        found = j
                        break
                if found < 0:
                    ids.append(key)
                    found = len(ids) - 1
                colmap.append(found)
                cmap[(d, m, r)] = found
    u = len(ids)

    pt = {}
    qt = {}
    for d in range(2, D + 1):
        for r in range(ranks[d]):
            pk = tuple(sorted(cmap[(d, m, r)] for m in range(d)))
            pt[pk] = pt.get(pk, 0) + 1
            qk = (d, cmap[(d, d - 1, r)], tuple(sorted(cmap[(d, m, r)] for m in range(d - 1))))
            qt[qk] = qt.get(qk, 0) + 1
    pterms = sorted(pt.items(), key=lambda kv: (len(kv[0]), kv[0]))
    qterms = sorted(qt.items(), key=lambda kv: kv[0])

    cs = PREC_BYTES[prec]
    split = None
    if mixed:
        Lm = None
        for base in (48, 80):
            c = base
            while c < De * N - 1:
                c *= 2
            if Lm is None or c < Lm:
                Lm = c
        if Lm < L:
            split = _mixed_split(Lm, u, cs)
            if split is not None:
                L, M = Lm, Lm // 2
    if split is not None:
        M1, M2, g = split
    else:
        lg = _log2_exact(M)
        M1 = 1 << ((lg + 1) // 2)
        M2 = M // M1
        while u * 2 * M2 * cs > 65536 and M1 < 2048:
            M1 *= 2
            M2 //= 2
        if M1 > 2048:
            raise Unsupported(f"no two-pass split for L={L}")
        if M2 < 2:
            raise Unsupported(f"u={u} distinct columns leave rows of one value at L={L}")
        g = min(M2, max(1, 1024 // M1))

    chunks = []
    if u * 2 * (M2 + M2 // 16) * cs + (M2 * cs if M2 <= 512 else 0) > 147456:
        cmax = 151552 // (2 * (M2 + M2 // 16) * cs)
        order = sorted(range(len(pterms)), key=lambda t: (tuple(sorted(set(pterms[t][0]))), t))
        cols, terms = set(), []
        for t in order:
            need = set(pterms[t][0])
            if len(need) > cmax:
                raise Unsupported(f"a gain term has {len(need)} distinct columns; a chunk holds {cmax}")
            if terms and len(cols | need) > cmax:
                chunks.append((sorted(cols), terms))
                cols, terms = set(), []
            cols |= need
            terms.append(t)
        if terms:
            chunks.append((sorted(cols), terms))

    flat = [L, M1, M2, g, u, len(pterms), len(qterms), De] + colmap
    for key, mult in pterms:
        flat += [len(key), mult] + list(key)
    for (d, km, others), mult in qterms:
        flat += [d, mult, km] + list(others)
    flat.append(len(chunks))
    for cols, terms in chunks:
        flat += [len(cols), len(terms)] + cols + terms
    return dict(L=L, M=M, M1=M1, M2=M2, g=g, u=u, De=De, colmap=colmap,
                pterms=pterms, qterms=qterms, chunks=chunks, flat=np.array(flat, dtype=np.int64))


def plan_tables_tt(D: int, N: int, tt: dict, prec: str = "fp64", mixed: bool = False):
    """The written rules for kernels in tensor-train form (Sec. 2): {d: cores},
    core m of shape (r_{m-1}, N, r_m).

    T1  Effective order and L as P1/P2 (De = largest d listed).
    T2  Column ids: scan d ascending, cores m = 1..d, a < r_{m-1}, b < r_m; the
        core column H^(m)[a, :, b] gets -1 when all its values are zero, else the
        id of the first earlier bitwise-equal column, else the next new id.
    T3  Split and tile as P6/P7 with u distinct columns (with the mixed-radix
        option: X2/X6/X7 first, as for CP kernels).  Unsupported when M2 > 512.
    T4  Chunks always (the chain runs in the chunked row pass): capacity as in
        P8, cores taken in scan order, a chunk taking the next core while the
        union of distinct non-negative ids stays within the capacity, else a
        new chunk starts with that core.  Unsupported if one core alone has
        more distinct ids than the capacity.

    Flat table: [L, M1, M2, g, u, T, K, De, d per term,
                 per core: term, m, r_in, r_out, ids[r_in r_out] (row-major),
                 nchunks, per chunk: ncols, ncores, ids, core indices]."""
    orders = sorted(tt)
    De = max(orders) if orders else 2
    L = 1
    while L < De * N - 1:
        L *= 2
    L = max(16, L)
    M = L // 2
    seen = []
    cores_rec = []       # (term, m, rin, rout, ids)
    for t, d in enumerate(orders):
        for m in range(1, d + 1):
            H = np.asarray(tt[d][m - 1], dtype=np.float64)
            rin, rout = H.shape[0], H.shape[2]
            ids = []
            for a in range(rin):
                for b in range(rout):
                    col = np.ascontiguousarray(H[a, :, b])
                    if not np.any(col != 0.0):
                        ids.append(-1)
                        continue
                    key = col.tobytes()
                    if key in seen:
                        ids.append(seen.index(key))
                    else:
                        seen.append(key)
                        ids.append(len(seen) - 1)
            cores_rec.append((t, m, rin, rout, ids))
    u = len(seen)
    cs = PREC_BYTES[prec]
    split = None
    if mixed:
        Lm = None
        for base in (48, 80):
            c = base
            while c < De * N - 1:
                c *= 2
            if Lm is None or c < Lm:
                Lm = c
        if Lm < L:
            split = _mixed_split(Lm, u, cs)
            if split is not None:
                L, M = Lm, Lm // 2
    if split is not None:
        M1, M2, g = split
    else:
        lg = _log2_exact(M)
        M1 = 1 << ((lg + 1) // 2)
        M2 = M // M1
        while u * 2 * M2 * cs > 65536 and M1 < 2048:
            M1 *= 2
            M2 //= 2
        if M1 > 2048 or M2 < 2:
            raise Unsupported(f"no two-pass split for L={L} with u={u}")
        g = min(M2, max(1, 1024 // M1))
    if M2 > 512:
        raise Unsupported("tensor-train chains need rows of at most 512 values")
    cmax = 151552 // (2 * (M2 + M2 // 16) * cs)
    chunks = []
    cols, cores = set(), []
    for k, rec in enumerate(cores_rec):
        need = {i for i in rec[4] if i >= 0}
        if len(need) > cmax:
            raise Unsupported(f"a core has {len(need)} distinct columns; a chunk holds {cmax}")
        if cores and len(cols | need) > cmax:
            chunks.append((sorted(cols), cores))
            cols, cores = set(), []
        cols |= need
        cores.append(k)
    if cores:
        chunks.append((sorted(cols), cores))
    flat = [L, M1, M2, g, u, len(orders), len(cores_rec), De] + list(orders)
    for (t, m, rin, rout, ids) in cores_rec:
        flat += [t, m, rin, rout] + ids
    flat.append(len(chunks))
    for cols, cores in chunks:
        flat += [len(cols), len(cores)] + cols + cores
    return dict(L=L, M1=M1, M2=M2, g=g, u=u, De=De, cores=cores_rec, chunks=chunks,
                flat=np.array(flat, dtype=np.int64))

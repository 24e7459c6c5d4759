"""Seeded synthetic alignment workloads (inputs only, no alignment arithmetic).

This module builds sequences, lengths and scoring schemes.  It is the only
code shared between the GPU path's tests/benchmark and the CPU oracle's tests:
both sides receive the same bytes from here.

Random numbers come from SplitMix64 used as a counter-based generator: draw n
of stream (seed, stream_id) is  mix(key + (n+1) * 0x9E3779B97F4A7C15)  with
key = mix(seed * 0x100000001B3 + stream_id) and mix() the SplitMix64 output
function (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014).  Draws are reproducible independent of NumPy's own
generators.  Uniform doubles use the top 53 bits; integers in [lo, hi] are
floor(u * (hi - lo + 1)) + lo.

Workloads (codes: DNA A,C,G,T = 0..3; protein = 0..19):
  nw_dna_1k      256 pairs, reference 1000 bp, query = reference with 10% edits
                 (substitution:insertion:deletion = 2:1:1); NW, +2/-4, open -4,
                 extend -2; full matrix + CIGAR.
  sw_protein     65,536 pairs, lengths lognormal (median 350, sigma 0.6) clipped
                 to [50, 2000] per side, 30% homologous (40% identity window);
                 symmetric seeded 20x20 matrix (diagonal U{4..11}, off-diagonal
                 U{-4..3}); SW, open -11, extend -1; score + end cell.
  band_long      2,048 pairs, reference U{10,000..100,000} bp, query with 12%
                 errors (insertion:deletion:substitution = 5:4:3); NW, +1/-2,
                 open -2, extend -1; static band half-width 256 + CIGAR.
  xdrop_ext      200,000 seed extensions (31 bp exact seed), each side of length
                 U{150..5,000} at divergence U[0.05, 0.25] (2:1:1) followed by
                 an unrelated random flank of ceil(0.1 L) bases; EXTEND + X-drop
                 X = 100, +2/-4, open -4, extend -2.  Both sides are stored as
                 sequences read away from the seed (the left side reversed).
  zdrop_ext      the xdrop_ext pairs (same seed, same bytes) under Z-drop with
                 Z = 100, so the two pruning rules are compared on one input.
  xdrop_cigar    the xdrop_ext pairs with a CIGAR per extension side (the
                 traceback through the X-drop region).
  edit_search    4,096 pairs of 2,000 bp at 5% divergence (sub:ins:del = 2:1:1),
                 unit edit costs, global; the score-major search schedule.
                 edit_pairs() builds the same kind of batch for any length and
                 divergence (the sizes and divergences of the paper's
                 edit-distance table) and penalties.
  affine_search  the edit_search shape (seed 707) under gap-affine penalties:
                 mismatch 4, gap open 6, extend 2.
"""
from dataclasses import dataclass, field

import numpy as np

GLOBAL, LOCAL, EXTEND = 0, 1, 2
FULL, BAND, XDROP, ZDROP, SEARCH = 0, 1, 2, 3, 4

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


class Stream:
    """Counter-based SplitMix64 stream; every call consumes fresh counters."""

    def __init__(self, seed, stream_id=0):
        with np.errstate(over="ignore"):
            k = np.uint64(seed) * np.uint64(0x100000001B3) + np.uint64(stream_id)
        self.key = _mix(np.array([k], dtype=np.uint64))[0]
        self.ctr = 0

    def u64(self, n):
        idx = np.arange(self.ctr + 1, self.ctr + 1 + n, dtype=np.uint64)
        self.ctr += n
        with np.errstate(over="ignore"):
            return _mix(self.key + idx * _GAMMA)

    def u64_at(self, start, n):
        """Draws start .. start+n-1 of the stream (does not move the counter)."""
        idx = np.arange(start + 1, start + 1 + n, dtype=np.uint64)
        with np.errstate(over="ignore"):
            return _mix(self.key + idx * _GAMMA)

    def uniform(self, n):
        return (self.u64(n) >> np.uint64(11)).astype(np.float64) * (1.0 / (1 << 53))

    def integers(self, lo, hi, n):
        """n integers uniform in [lo, hi] (inclusive), as int64."""
        span = np.asarray(hi, dtype=np.int64) - np.asarray(lo, dtype=np.int64) + 1
        u = self.uniform(n)
        return (np.floor(u * span).astype(np.int64) + lo).astype(np.int64)

    def normal(self, n):
        """Box-Muller standard normals."""
        u1 = self.uniform(n)
        u2 = self.uniform(n)
        u1 = np.where(u1 <= 0.0, 1.0 / (1 << 53), u1)
        return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


@dataclass
class Batch:
    """A batch of pairs in the layout the library consumes."""
    name: str
    q: np.ndarray          # uint8 codes, concatenated
    q_off: np.ndarray      # int64
    q_len: np.ndarray      # int32
    r: np.ndarray
    r_off: np.ndarray
    r_len: np.ndarray
    matrix: np.ndarray     # int32 [alphabet, alphabet]
    gap_open: int
    gap_extend: int
    mode: int
    prune: int
    band_w: int = 0
    xdrop: int = 0
    want_cigar: bool = False
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.q_len.size)

    @property
    def alphabet(self):
        return int(self.matrix.shape[0])

    def pair(self, p):
        qs = self.q[self.q_off[p]: self.q_off[p] + self.q_len[p]]
        rs = self.r[self.r_off[p]: self.r_off[p] + self.r_len[p]]
        return qs, rs

    def subset(self, idx, name=None):
        idx = np.asarray(idx, dtype=np.int64)
        qs = [self.pair(int(p))[0] for p in idx]
        rs = [self.pair(int(p))[1] for p in idx]
        b = pack_pairs(qs, rs, self.matrix, self.gap_open, self.gap_extend,
                       self.mode, self.prune, self.band_w, self.xdrop,
                       self.want_cigar, name or self.name + "_subset")
        b.meta = dict(self.meta, subset_of=self.name, subset_idx=idx)
        return b


def pack_pairs(qs, rs, matrix, gap_open, gap_extend, mode, prune, band_w=0,
               xdrop=0, want_cigar=False, name="pairs"):
    ql = np.array([len(x) for x in qs], dtype=np.int32)
    rl = np.array([len(x) for x in rs], dtype=np.int32)
    qo = np.zeros(len(qs), dtype=np.int64)
    ro = np.zeros(len(rs), dtype=np.int64)
    if len(qs) > 1:
        qo[1:] = np.cumsum(ql[:-1], dtype=np.int64)
        ro[1:] = np.cumsum(rl[:-1], dtype=np.int64)
    q = (np.concatenate([np.asarray(x, dtype=np.uint8) for x in qs])
         if len(qs) and ql.sum() else np.zeros(0, dtype=np.uint8))
    r = (np.concatenate([np.asarray(x, dtype=np.uint8) for x in rs])
         if len(rs) and rl.sum() else np.zeros(0, dtype=np.uint8))
    return Batch(name, q, qo, ql, r, ro, rl, np.ascontiguousarray(matrix, dtype=np.int32),
                 int(gap_open), int(gap_extend), int(mode), int(prune), int(band_w),
                 int(xdrop), bool(want_cigar))


def dna_matrix(match, mismatch):
    m = np.full((4, 4), mismatch, dtype=np.int32)
    np.fill_diagonal(m, match)
    return m


def protein_matrix(seed):
    """Symmetric 20x20: S[a][a] ~ U{4..11}; for a < b, S[a][b] = S[b][a] ~
    U{-4..3}, drawn in the order a = 0..19 (diagonal first), then b = a+1..19."""
    st = Stream(seed, 99)
    m = np.zeros((20, 20), dtype=np.int32)
    for a in range(20):
        m[a, a] = st.integers(4, 11, 1)[0]
        for b in range(a + 1, 20):
            v = st.integers(-4, 3, 1)[0]
            m[a, b] = v
            m[b, a] = v
    return m


def mutate(ref, rate, w_sub, w_ins, w_del, alphabet, st):
    """Walk ref; each base is edited with probability ``rate``, the edit type
    drawn with weights sub:ins:del.  sub = a uniformly random different code;
    ins = copy the base, then insert one random code; del = drop the base."""
    n = ref.size
    u_edit = st.uniform(n)
    u_type = st.uniform(n)
    u_c1 = st.uniform(n)
    u_c2 = st.uniform(n)
    tot = float(w_sub + w_ins + w_del)
    edit = u_edit < rate
    t = u_type * tot
    is_sub = edit & (t < w_sub)
    is_ins = edit & (t >= w_sub) & (t < w_sub + w_ins)
    is_del = edit & (t >= w_sub + w_ins)
    first = ref.astype(np.int64).copy()
    shift = 1 + np.floor(u_c1 * (alphabet - 1)).astype(np.int64)
    first[is_sub] = (first[is_sub] + shift[is_sub]) % alphabet
    second = np.floor(u_c2 * alphabet).astype(np.int64)
    cnt = np.ones(n, dtype=np.int64)
    cnt[is_ins] = 2
    cnt[is_del] = 0
    out = np.empty(int(cnt.sum()), dtype=np.uint8)
    starts = np.cumsum(cnt) - cnt
    keep = cnt >= 1
    out[starts[keep]] = first[keep]
    out[starts[is_ins] + 1] = second[is_ins]
    return out


def random_codes(st, n, alphabet):
    return np.floor(st.uniform(n) * alphabet).astype(np.uint8)


# ---------------------------------------------------------------- configs
def nw_dna_1k(n=256, ref_len=1000, seed=101):
    st = Stream(seed, 1)
    qs, rs = [], []
    for _ in range(n):
        ref = random_codes(st, ref_len, 4)
        qry = mutate(ref, 0.10, 2, 1, 1, 4, st)
        qs.append(qry)
        rs.append(ref)
    b = pack_pairs(qs, rs, dna_matrix(2, -4), -4, -2, GLOBAL, FULL,
                   want_cigar=True, name="nw_dna_1k")
    b.meta = dict(seed=seed)
    return b


def _lognormal_lengths(st, n, median, sigma, lo, hi):
    z = st.normal(n)
    x = np.exp(np.log(median) + sigma * z)
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def sw_protein(n=65536, seed=202, sigma=0.6, homolog_frac=0.3, identity=0.4):
    st = Stream(seed, 2)
    mat = protein_matrix(seed)
    M = _lognormal_lengths(st, n, 350.0, sigma, 50, 2000)
    N = _lognormal_lengths(st, n, 350.0, sigma, 50, 2000)
    hom = st.uniform(n) < homolog_frac
    q_all = random_codes(st, int(M.sum()), 20)
    r_all = random_codes(st, int(N.sum()), 20)
    qo = np.zeros(n, dtype=np.int64)
    ro = np.zeros(n, dtype=np.int64)
    qo[1:] = np.cumsum(M[:-1])
    ro[1:] = np.cumsum(N[:-1])
    # homologous pairs: a window of length min(M,N) at random offsets in both;
    # the query window copies the reference window, keeping each residue with
    # probability `identity`, else a uniformly random different residue
    idx = np.nonzero(hom)[0]
    W = np.minimum(M[idx], N[idx])
    uq = st.uniform(idx.size)
    ur = st.uniform(idx.size)
    oq = np.floor(uq * (M[idx] - W + 1)).astype(np.int64)
    orr = np.floor(ur * (N[idx] - W + 1)).astype(np.int64)
    tot = int(W.sum())
    keep = st.uniform(tot) < identity
    shift = 1 + np.floor(st.uniform(tot) * 19).astype(np.int64)
    src = np.concatenate([ro[p] + o + np.arange(w) for p, o, w in zip(idx, orr, W)]) \
        if idx.size else np.zeros(0, dtype=np.int64)
    dst = np.concatenate([qo[p] + o + np.arange(w) for p, o, w in zip(idx, oq, W)]) \
        if idx.size else np.zeros(0, dtype=np.int64)
    base = r_all[src].astype(np.int64)
    q_all[dst] = np.where(keep, base, (base + shift) % 20).astype(np.uint8)
    b = Batch("sw_protein", q_all, qo, M.astype(np.int32), r_all, ro, N.astype(np.int32),
              mat, -11, -1, LOCAL, FULL)
    b.meta = dict(seed=seed, sigma=sigma, homologous=hom)
    return b


def _segments(lengths):
    """Start offsets of consecutive segments with the given lengths."""
    off = np.zeros(len(lengths), dtype=np.int64)
    if len(lengths) > 1:
        off[1:] = np.cumsum(lengths[:-1])
    return off


def _dna_sides_chunk(x, y, L, rate, flank, w_sub, w_ins, w_del):
    """One chunk of _dna_sides: x holds one draw per reference base, y one per
    flank base; returns (q, q_len, r, r_len) for these sides, concatenated."""
    ns = L.size
    ref = (x & np.uint64(3)).astype(np.uint8)
    u_edit = (x >> np.uint64(40)).astype(np.float64) * (1.0 / (1 << 24))
    u_type = ((x >> np.uint64(2)) & np.uint64(0xFFFFFF)).astype(np.float64) * (1.0 / (1 << 24))
    ins_code = ((x >> np.uint64(26)) & np.uint64(3)).astype(np.uint8)
    u_sub = ((x >> np.uint64(28)) & np.uint64(0xFFF)).astype(np.float64) * (1.0 / (1 << 12))
    tot = float(w_sub + w_ins + w_del)
    edit = u_edit < np.repeat(rate, L)
    t = u_type * tot
    is_sub = edit & (t < w_sub)
    is_ins = edit & (t >= w_sub) & (t < w_sub + w_ins)
    is_del = edit & (t >= w_sub + w_ins)
    first = ref.copy()
    shift = (1 + np.floor(u_sub * 3)).astype(np.uint8)
    first[is_sub] = (first[is_sub] + shift[is_sub]) % 4
    cnt = np.ones(ref.size, dtype=np.int64)
    cnt[is_ins] = 2
    cnt[is_del] = 0
    starts = np.cumsum(cnt) - cnt
    qext = np.empty(int(cnt.sum()), dtype=np.uint8)
    keep = cnt >= 1
    qext[starts[keep]] = first[keep]
    qext[starts[is_ins] + 1] = ins_code[is_ins]
    seg = _segments(L)
    ccnt = np.concatenate([[0], np.cumsum(cnt)])
    qlen_ext = ccnt[seg + L] - ccnt[seg]
    rfl = (y & np.uint64(3)).astype(np.uint8)
    qfl = ((y >> np.uint64(2)) & np.uint64(3)).astype(np.uint8)

    def join(a, a_len, f, f_len):
        out_len = a_len + f_len
        out = np.empty(int(out_len.sum()), dtype=np.uint8)
        o = _segments(out_len)
        ia = np.arange(a.size, dtype=np.int64) - np.repeat(_segments(a_len), a_len)
        out[np.repeat(o, a_len) + ia] = a
        jf = np.arange(f.size, dtype=np.int64) - np.repeat(_segments(f_len), f_len)
        out[np.repeat(o + a_len, f_len) + jf] = f
        return out, out_len

    r, r_len = join(ref, L, rfl, flank)
    q, q_len = join(qext, qlen_ext, qfl, flank)
    return q, q_len, r, r_len


def _dna_sides(seed, stream_id, L, rate, w_sub, w_ins, w_del, flank=None,
               chunk_bases=1 << 22, threads=8):
    """DNA pairs with random reference r_p (length L[p]) and query q_p = r_p
    edited per base with probability rate[p] (types weighted sub:ins:del as in
    mutate()), each followed by an unrelated random flank of flank[p] bases.

    One 64-bit draw per reference base from stream (seed, stream_id) fixes the
    base (bits 0-1), the edit type (bits 2-25 as a uniform), the inserted base
    (bits 26-27), the substitution offset 1 + floor(3u) (bits 28-39) and the
    edit decision (bits 40-63 as a uniform); one draw per flank position from
    stream (seed, stream_id + 1) gives the reference (bits 0-1) and query
    (bits 2-3) flank bases.  Draws are indexed by absolute base position, so
    the output does not depend on chunking or threads."""
    from concurrent.futures import ThreadPoolExecutor
    L = np.asarray(L, dtype=np.int64)
    ns = L.size
    rate = np.broadcast_to(np.asarray(rate, dtype=np.float64), (ns,))
    flank = np.zeros(ns, np.int64) if flank is None else np.asarray(flank, np.int64)
    cumL = np.concatenate([[0], np.cumsum(L)])
    cumF = np.concatenate([[0], np.cumsum(flank)])
    bounds = [0]
    while bounds[-1] < ns:
        s0 = bounds[-1]
        s1 = int(np.searchsorted(cumL, cumL[s0] + chunk_bases, side="right")) - 1
        bounds.append(min(ns, max(s1, s0 + 1)))
    sx, sy = Stream(seed, stream_id), Stream(seed, stream_id + 1)

    def work(c):
        s0, s1 = bounds[c], bounds[c + 1]
        x = sx.u64_at(int(cumL[s0]), int(cumL[s1] - cumL[s0]))
        y = sy.u64_at(int(cumF[s0]), int(cumF[s1] - cumF[s0]))
        return _dna_sides_chunk(x, y, L[s0:s1], rate[s0:s1], flank[s0:s1],
                                w_sub, w_ins, w_del)

    with ThreadPoolExecutor(max_workers=threads) as ex:
        parts = list(ex.map(work, range(len(bounds) - 1)))
    q = np.concatenate([p[0] for p in parts]) if parts else np.zeros(0, np.uint8)
    q_len = np.concatenate([p[1] for p in parts]) if parts else np.zeros(0, np.int64)
    r = np.concatenate([p[2] for p in parts]) if parts else np.zeros(0, np.uint8)
    r_len = np.concatenate([p[3] for p in parts]) if parts else np.zeros(0, np.int64)
    return q, _segments(q_len), q_len.astype(np.int32), r, _segments(r_len), r_len.astype(np.int32)


def band_long(n=2048, seed=303, min_len=10000, max_len=100000, band_w=256):
    st = Stream(seed, 3)
    L = st.integers(min_len, max_len, n)
    q, qo, ql, r, ro, rl = _dna_sides(seed, 30, L, 0.12, 3, 5, 4)
    b = Batch("band_long", q, qo, ql, r, ro, rl, dna_matrix(1, -2), -2, -1, GLOBAL, BAND,
              band_w=band_w, want_cigar=True)
    b.meta = dict(seed=seed)
    return b


def xdrop_ext(n=200000, seed=404, min_len=150, max_len=5000, xdrop=100, seed_len=31):
    """2n extension problems: entries [0, n) are left sides, [n, 2n) right
    sides of the same n seeds.  meta['seed_score'] is the exact seed's score."""
    st = Stream(seed, 4)
    ns = 2 * n
    L = st.integers(min_len, max_len, ns)
    div = 0.05 + 0.20 * st.uniform(ns)
    flank = np.ceil(0.1 * L).astype(np.int64)
    seeds = random_codes(st, n * seed_len, 4).reshape(n, seed_len)
    q, qo, ql, r, ro, rl = _dna_sides(seed, 40, L, div, 2, 1, 1, flank=flank)
    b = Batch("xdrop_ext", q, qo, ql, r, ro, rl, dna_matrix(2, -4), -4, -2, EXTEND, XDROP,
              xdrop=xdrop)
    b.meta = dict(seed=seed, n_ext=n, seed_len=seed_len, seed_score=2 * seed_len,
                  seeds=seeds, L=L, div=div)
    return b


def zdrop_ext(n=200000, seed=404, min_len=150, max_len=5000, zdrop=100, seed_len=31):
    """The xdrop_ext extension problems under Z-drop with threshold Z."""
    b = xdrop_ext(n=n, seed=seed, min_len=min_len, max_len=max_len, xdrop=zdrop,
                  seed_len=seed_len)
    b.name = "zdrop_ext"
    b.prune = ZDROP
    return b


def xdrop_cigar(n=200000, seed=404, min_len=150, max_len=5000, xdrop=100, seed_len=31):
    """The xdrop_ext extension problems with a CIGAR per side."""
    b = xdrop_ext(n=n, seed=seed, min_len=min_len, max_len=max_len, xdrop=xdrop,
                  seed_len=seed_len)
    b.name = "xdrop_cigar"
    b.want_cigar = True
    return b


def edit_pairs(n, length, div, seed, prune=SEARCH, name=None, pen=(1, 0, 1)):
    """n pairs for edit distance: a uniform ACGT reference of `length`
    bases and a query that is the reference with per-base edits at rate
    `div` (substitution:insertion:deletion = 2:1:1).  `pen` = (mismatch x,
    gap open o, gap extend e) penalties, scored as (0, -x, -o, -e); the
    default is unit edit costs."""
    st = Stream(seed, 6)
    qs, rs = [], []
    for _ in range(n):
        ref = random_codes(st, length, 4)
        qs.append(mutate(ref, div, 2, 1, 1, 4, st))
        rs.append(ref)
    x, o, e = pen
    b = pack_pairs(qs, rs, dna_matrix(0, -x), -o, -e, GLOBAL, prune,
                   name=name or f"edit_{length}_{div}")
    b.meta = dict(seed=seed, length=length, div=div, pen=pen)
    return b


def edit_search(n=4096, length=2000, div=0.05, seed=606):
    return edit_pairs(n, length, div, seed, name="edit_search")


def affine_search(n=4096, length=2000, div=0.05, seed=707, pen=(4, 6, 2)):
    """The edit_search shape under gap-affine penalties (mismatch 4, open 6,
    extend 2)."""
    return edit_pairs(n, length, div, seed, name="affine_search", pen=pen)


@dataclass
class FoldBatch:
    """A batch of RNA sequences for the folding recurrence (codes A, C, G, U =
    0..3), with its pairing table and pruning parameters."""
    name: str
    x: np.ndarray        # uint8 codes, concatenated
    off: np.ndarray      # int64
    length: np.ndarray   # int32
    pair: np.ndarray     # int32 [4, 4] pairing scores
    min_loop: int = 0
    xdrop: int = -1      # < 0: unpruned
    warmup: int = 15
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.length.size)

    def seq(self, p):
        o = int(self.off[p])
        return self.x[o: o + int(self.length[p])]

    def subset(self, idx, name=None):
        xs = [self.seq(int(p)) for p in np.asarray(idx, dtype=np.int64)]
        return pack_fold(xs, self.pair, self.min_loop, self.xdrop, self.warmup,
                         name or self.name + "_subset")

    def with_params(self, **kw):
        b = FoldBatch(self.name, self.x, self.off, self.length, self.pair, self.min_loop,
                      self.xdrop, self.warmup, dict(self.meta))
        for k, v in kw.items():
            setattr(b, k, v)
        return b


def pack_fold(xs, pair, min_loop=0, xdrop=-1, warmup=15, name="fold"):
    length = np.array([len(x) for x in xs], dtype=np.int32)
    off = np.zeros(len(xs), dtype=np.int64)
    if len(xs) > 1:
        off[1:] = np.cumsum(length[:-1], dtype=np.int64)
    x = (np.concatenate([np.asarray(v, dtype=np.uint8) for v in xs]) if xs
         else np.zeros(0, dtype=np.uint8))
    return FoldBatch(name, x, off, length, np.asarray(pair, dtype=np.int32).reshape(4, 4),
                     int(min_loop), int(xdrop), int(warmup))


def rna_pair_table():
    """Pairing scores: one point per Watson-Crick pair (A-U, C-G) and per G-U
    wobble pair, symmetric; every other pair 0."""
    P = np.zeros((4, 4), dtype=np.int32)
    for a, b in ((0, 3), (1, 2), (2, 3)):
        P[a, b] = P[b, a] = 1
    return P


def rna_fold(n=4096, seed=808, min_len=76, max_len=500, xdrop=2, warmup=15, min_loop=3):
    """Seeded synthetic RNA: n sequences of i.i.d. uniform A, C, G, U with
    lengths uniform in [min_len, max_len] (the span of RNA lengths the folding
    experiment uses), pairing table rna_pair_table(), minimum hairpin loop
    min_loop, X-drop threshold xdrop (< 0: unpruned) after `warmup` spans."""
    st = Stream(seed, 1)
    lens = st.integers(min_len, max_len, n).astype(np.int32)
    codes = (st.u64(int(lens.sum())) & np.uint64(3)).astype(np.uint8)
    off = np.zeros(n, dtype=np.int64)
    if n > 1:
        off[1:] = np.cumsum(lens[:-1], dtype=np.int64)
    b = FoldBatch(f"rna_fold_x{xdrop}", codes, off, lens, rna_pair_table(), int(min_loop),
                  int(xdrop), int(warmup))
    b.meta = dict(seed=seed, min_len=min_len, max_len=max_len)
    return b


WORKLOADS = {
    "nw_dna_1k": nw_dna_1k,
    "sw_protein": sw_protein,
    "band_long": band_long,
    "xdrop_ext": xdrop_ext,
    "zdrop_ext": zdrop_ext,
    "xdrop_cigar": xdrop_cigar,
    "edit_search": edit_search,
    "affine_search": affine_search,
}


def serving_requests(n_req, qps, seed=505, mix=(0.4, 0.3, 0.1, 0.2),
                     scale_long=1.0):
    """Poisson arrivals (exponential gaps) of single-pair requests drawn from the
    four workloads above in proportions ``mix``.  Returns (arrival_s, kinds,
    batches) where batches[k] is a Batch holding that kind's requests in order.
    ``scale_long`` < 1 shortens band_long requests (for small test runs)."""
    st = Stream(seed, 5)
    gaps = -np.log(np.maximum(st.uniform(n_req), 1e-300)) / float(qps)
    arrival = np.cumsum(gaps)
    u = st.uniform(n_req)
    cum = np.cumsum(np.asarray(mix, dtype=np.float64))
    kinds = np.searchsorted(cum / cum[-1], u, side="right").astype(np.int64)
    kinds = np.minimum(kinds, 3)
    counts = [int((kinds == k).sum()) for k in range(4)]
    batches = [
        nw_dna_1k(n=max(counts[0], 1), seed=seed + 1),
        sw_protein(n=max(counts[1], 1), seed=seed + 2),
        band_long(n=max(counts[2], 1), seed=seed + 3,
                  min_len=max(64, int(10000 * scale_long)),
                  max_len=max(128, int(100000 * scale_long))),
        xdrop_ext(n=max((counts[3] + 1) // 2, 1), seed=seed + 4),
    ]
    return arrival, kinds, batches

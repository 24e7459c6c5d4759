"""Brute-force enumeration of alignments, independent of any recurrence.

Used only to pin the oracle.  Every alignment of q (rows) against r (columns)
is a monotone path of moves: 'M' (diagonal, consumes q_i and r_j), 'I'
(vertical, consumes q_i), 'D' (horizontal, consumes r_j).  Its score is the sum
of substitution scores of the 'M' moves plus, for every maximal run of the same
gap move, open + L*extend (Gotoh's affine gap cost; an I-run directly followed
by a D-run is two runs, each opened).

``state_paths`` enumerates the finer objects the traceback chooses between:
paths through the three states H/E/F where each gap step is labelled open or
extend.  They are used to pin the traceback tie-break.
"""
import itertools


def move_paths(M, N):
    """All move strings from (0,0) to (M,N)."""
    out = []

    def rec(i, j, acc):
        if i == M and j == N:
            out.append("".join(acc))
            return
        if i < M and j < N:
            acc.append("M"); rec(i + 1, j + 1, acc); acc.pop()
        if i < M:
            acc.append("I"); rec(i + 1, j, acc); acc.pop()
        if j < N:
            acc.append("D"); rec(i, j + 1, acc); acc.pop()

    rec(0, 0, [])
    return out


def path_cells(moves, i0=0, j0=0):
    cells = [(i0, j0)]
    i, j = i0, j0
    for mv in moves:
        if mv == "M":
            i += 1; j += 1
        elif mv == "I":
            i += 1
        else:
            j += 1
        cells.append((i, j))
    return cells


def score_moves(moves, q, r, S, o, e, i0=0, j0=0):
    i, j = i0, j0
    total = 0
    for mv, grp in itertools.groupby(moves):
        L = len(list(grp))
        if mv == "M":
            for _ in range(L):
                total += S[q[i]][r[j]]
                i += 1; j += 1
        elif mv == "I":
            total += o + L * e
            i += L
        else:
            total += o + L * e
            j += L
    return total


def global_best(q, r, S, o, e, allowed=None):
    """Max over all alignments of q and r (optionally only paths whose cells
    all satisfy ``allowed(i, j)``); None when no path is allowed."""
    best = None
    for p in move_paths(len(q), len(r)):
        if allowed is not None and not all(allowed(i, j) for i, j in path_cells(p)):
            continue
        sc = score_moves(p, q, r, S, o, e)
        if best is None or sc > best:
            best = sc
    return best


def local_best(q, r, S, o, e):
    """Smith-Waterman by enumeration: max over every pair of substrings
    (empty allowed, scoring 0).  Returns (score, end_i, end_j) with the end
    order: higher score, then smaller i, then smaller j; score 0 ends at (0,0)."""
    M, N = len(q), len(r)
    best = (0, 0, 0)
    for a in range(M + 1):
        for b in range(a + 1, M + 1):
            for c in range(N + 1):
                for d in range(c + 1, N + 1):
                    g = global_best(q[a:b], r[c:d], S, o, e)
                    cand = (g, b, d)
                    if _better(cand, best):
                        best = cand
    return best


def extend_best(q, r, S, o, e):
    """Seed extension by enumeration: max over every pair of prefixes (the
    empty pair scores 0).  Same end order as local_best."""
    M, N = len(q), len(r)
    best = (0, 0, 0)
    for b in range(M + 1):
        for d in range(N + 1):
            if b == 0 and d == 0:
                continue
            g = global_best(q[:b], r[:d], S, o, e)
            if _better((g, b, d), best):
                best = (g, b, d)
    return best


def _better(a, b):
    if a[0] != b[0]:
        return a[0] > b[0]
    if a[1] != b[1]:
        return a[1] < b[1]
    return a[2] < b[2]


# ---------------------------------------------------------------- state paths
# Labels, compared position by position walking back from the end cell:
#   in state H: stop(LOCAL) 0 < diag 1 < E 2 < F 3;   in E or F: open 0 < extend 1.
def state_paths(q, r, S, o, e, end, local):
    """Enumerate every state path ending at cell ``end`` in state H.
    Yields (value, labels, ops_forward, begin_cell)."""
    res = []

    def rec(i, j, st, val, labels, ops):
        if st == "H":
            if local:
                # a local alignment may start here (value of the rest is 0)
                res.append((val, labels + [0], ops[::-1], (i, j)))
                if i == 0 or j == 0:
                    return
            else:
                if i == 0 and j == 0:
                    res.append((val, labels, ops[::-1], (0, 0)))
                    return
                if i == 0:   # boundary row: one gap run back to (0,0)
                    res.append((val + o + j * e, labels, (ops + ["D"] * j)[::-1], (0, 0)))
                    return
                if j == 0:
                    res.append((val + o + i * e, labels, (ops + ["I"] * i)[::-1], (0, 0)))
                    return
            sub = S[q[i - 1]][r[j - 1]]
            rec(i - 1, j - 1, "H", val + sub, labels + [1],
                ops + ["=" if q[i - 1] == r[j - 1] else "X"])
            rec(i, j, "E", val, labels + [2], ops)
            rec(i, j, "F", val, labels + [3], ops)
        elif st == "E":            # D move consumes r_j
            rec(i, j - 1, "H", val + o + e, labels + [0], ops + ["D"])
            if j - 1 >= 1:
                rec(i, j - 1, "E", val + e, labels + [1], ops + ["D"])
        else:                      # F: I move consumes q_i
            rec(i - 1, j, "H", val + o + e, labels + [0], ops + ["I"])
            if i - 1 >= 1:
                rec(i - 1, j, "F", val + e, labels + [1], ops + ["I"])

    rec(end[0], end[1], "H", 0, [], [])
    return res


def run_length(ops):
    return [(op, len(list(g))) for op, g in itertools.groupby(ops)]


def op_cells(ops, begin=(0, 0)):
    """Cells visited by forward CIGAR ops ('=', 'X', 'I', 'D') from ``begin``."""
    return path_cells(["M" if op in "=X" else op for op in ops], *begin)


def preferred_path(q, r, S, o, e, end, local, allowed=None):
    """Among the optimal state paths ending at ``end``, the one with the
    lexicographically smallest label sequence.  With ``allowed``, only paths
    whose every cell satisfies allowed(i, j) take part.  Returns (value,
    cigar, begin)."""
    paths = state_paths(q, r, S, o, e, end, local)
    if allowed is not None:
        paths = [p for p in paths if all(allowed(i, j) for i, j in op_cells(p[2], p[3]))]
    best = max(p[0] for p in paths)
    opt = [p for p in paths if p[0] == best]
    opt.sort(key=lambda p: p[1])
    v, _, ops, begin = opt[0]
    return v, run_length(ops), begin

"""Helpers comparing GPU results with the CPU oracle, element by element."""
import os

import numpy as np

import oracle

INT32_MIN = -(1 << 31)
# X-drop / Z-drop with CIGAR: the widest candidate span (in diagonals) of the
# antidiagonals up to the end cell that the traceback window holds; a wider
# pair reports CIGAR_CAP with score, end cell and cells still exact.
DYN_CIGAR_SPAN = 250


SEARCH = 4  # the library's score-major search schedule (edit distance, gap-affine penalties)


def search_cells(S, M, N, e=1):
    """(score, diagonal) entries of the search domain for smallest penalty S
    and gap-extension penalty e: diagonals max(-s//e, -M) .. min(s//e, N) for
    s = 0 .. S (edit distance: e = 1)."""
    return sum(min(s // e, N) + min(s // e, M) + 1 for s in range(S + 1))


def oracle_batch(batch, want_cigar=None, nthreads=None):
    """The oracle's results for a batch.  A search batch is checked against
    the definition it computes: the full-matrix global alignment under the
    same scoring (unit edit costs or gap-affine penalties)."""
    wc = batch.want_cigar if want_cigar is None else want_cigar
    prune = oracle.FULL if batch.prune == SEARCH else batch.prune
    return oracle.align_batch(batch.matrix, batch.gap_open, batch.gap_extend,
                              batch.q, batch.q_off, batch.q_len,
                              batch.r, batch.r_off, batch.r_len,
                              mode=batch.mode, prune=prune, band_w=batch.band_w,
                              xdrop=batch.xdrop, want_cigar=wc,
                              nthreads=nthreads or min(16, os.cpu_count() or 1))


def compare(batch, gres, gcig, ores, check_cigar=None, idx=None, max_report=8):
    """Return a list of mismatch descriptions (empty when bit-exact).
    ``idx`` maps GPU result rows to oracle rows (default: identity)."""
    if check_cigar is None:
        check_cigar = batch.want_cigar
    bad = []
    n = len(gres)
    for k in range(n):
        p = k if idx is None else int(idx[k])
        g = gres[k]
        so, sg = int(ores["status"][p]), int(g["status"])
        if (check_cigar and batch.prune in (oracle.XDROP, oracle.ZDROP) and so == oracle.OK
                and int(ores["span"][p]) > DYN_CIGAR_SPAN):
            so = oracle.CIGAR_CAP
        if so != sg:
            bad.append(f"pair {p}: status gpu {sg} oracle {so}")
            continue
        if so == oracle.BAD_SYMBOL:
            continue
        exp_cells = int(ores["cells"][p])
        if batch.prune == SEARCH:
            exp_cells = search_cells(-int(ores["score"][p]), int(batch.q_len[p]),
                                     int(batch.r_len[p]), -int(batch.gap_extend))
        exp = (int(ores["score"][p]), int(ores["q_end"][p]), int(ores["r_end"][p]), exp_cells)
        got = (int(g["score"]), int(g["q_end"]), int(g["r_end"]), int(g["cells"]))
        if exp != got:
            bad.append(f"pair {p} (M={batch.q_len[p]}, N={batch.r_len[p]}): "
                       f"gpu (score,qe,re,cells)={got} oracle={exp}")
        if check_cigar and so == oracle.OK:
            ob = (int(ores["q_begin"][p]), int(ores["r_begin"][p]))
            gb = (int(g["q_begin"]), int(g["r_begin"]))
            oc = ores["cigar"][ores["cigar_off"][p]: ores["cigar_off"][p] + ores["cigar_len"][p]]
            gc = gcig[k]
            if ob != gb or not np.array_equal(np.asarray(oc, dtype=np.uint32),
                                              np.asarray(gc, dtype=np.uint32)):
                bad.append(f"pair {p}: cigar/begin differ (gpu begin {gb}, oracle {ob}, "
                           f"len gpu {len(gc)} oracle {len(oc)})")
        if len(bad) >= max_report:
            break
    return bad

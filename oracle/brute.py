"""Literal enumerators used to pin the C oracle (test infrastructure only).

* ``tally2`` / ``tally3`` follow the worked examples of Sec. 2.1 (Fig. 1) and
  Sec. 2.2 (Fig. 2) word for word: for each field, every allele of one entry
  is paired with every allele of the other entry(ies), and each resulting
  tuple of allele values is tallied.  Entries equal to the missing marker
  (1,0) take part in no tuple.
* ``x_matrix`` / ``tally3_via_x`` follow the paper's 3-way construction of
  Sec. 3.2: the modified matrices X_{j,xi} of Table 1, the tally operator
  that discards null entries, and the eight mapping identities that rebuild
  the 3-way tables from three restricted 2-way tallies.

Pure Python loops: only for tiny inputs.
"""
from __future__ import annotations

import numpy as np

MISSING = (1, 0)
NULL = (1, 0)  # Table 1's "null" indicator value


def unpack_codes(v: np.ndarray, n_f: int) -> np.ndarray:
    """Codes [n_v, n_f] from the packed rows (field q at bits 2(q%4))."""
    v = np.asarray(v, dtype=np.uint8)
    q = np.arange(n_f)
    return (v[:, q // 4] >> (2 * (q % 4)).astype(np.uint8)) & 3


def allele_pair(code: int):
    """The entry as an allele pair (high bit, low bit)."""
    return ((int(code) >> 1) & 1, int(code) & 1)


def tally2(codes_i, codes_j):
    """2x2 table [a][b] of allele co-occurrences of two vectors of codes."""
    t = np.zeros((2, 2), dtype=np.int64)
    for ci, cj in zip(codes_i, codes_j):
        ei, ej = allele_pair(ci), allele_pair(cj)
        if ei == MISSING or ej == MISSING:
            continue
        for x in ei:
            for y in ej:
                t[x, y] += 1
    return t


def tally3(codes_i, codes_j, codes_k):
    """2x2x2 table [a][b][c] of allele co-occurrences of three vectors."""
    t = np.zeros((2, 2, 2), dtype=np.int64)
    for ci, cj, ck in zip(codes_i, codes_j, codes_k):
        ei, ej, ek = allele_pair(ci), allele_pair(cj), allele_pair(ck)
        if MISSING in (ei, ej, ek):
            continue
        for x in ei:
            for y in ej:
                for z in ek:
                    t[x, y, z] += 1
    return t


def all_pairs(codes: np.ndarray) -> np.ndarray:
    """[P, 4] tables for all i<j in lexicographic order, entry 2a+b."""
    n = codes.shape[0]
    out = [tally2(codes[i], codes[j]).reshape(4) for i in range(n) for j in range(i + 1, n)]
    return np.array(out, dtype=np.int64).reshape(-1, 4)


def all_triples(codes: np.ndarray) -> np.ndarray:
    """[T, 8] tables for all i<j<k in lexicographic order, entry 4a+2b+c."""
    n = codes.shape[0]
    out = [tally3(codes[i], codes[j], codes[k]).reshape(8)
           for i in range(n) for j in range(i + 1, n) for k in range(j + 1, n)]
    return np.array(out, dtype=np.int64).reshape(-1, 8)


# ---------------------------------------------------------------------------
# The 3-way construction of Sec. 3.2.
# ---------------------------------------------------------------------------

GENOTYPES = {1: (0, 0), 2: (0, 1), 3: (1, 1)}  # xi -> genotype of V's entry


def _canon(e):
    """(1,0) and (0,1) tally identically; the paper folds (1,0) into (0,1)
    when the data has no missing entries."""
    return (0, 1) if e == (1, 0) else e


def x_entry(v_entry, vj_entry, xi: int, missing_aware: bool = True):
    """Entry of X_{j,xi}: v_j's entry where V's entry equals genotype xi, the
    null indicator elsewhere.  With ``missing_aware`` a missing entry of V or
    of v_j yields null (the paper's sketch for missing data)."""
    if missing_aware and (v_entry == MISSING or vj_entry == MISSING):
        return NULL
    if not missing_aware:
        v_entry, vj_entry = _canon(v_entry), _canon(vj_entry)
    return vj_entry if v_entry == GENOTYPES[xi] else NULL


def x_matrix(codes: np.ndarray, j: int, xi: int, missing_aware: bool = True):
    """X_{j,xi} as a list of columns (one per vector p) of allele pairs."""
    n_v, n_f = codes.shape
    return [[x_entry(allele_pair(codes[p, q]), allele_pair(codes[j, q]), xi, missing_aware)
             for q in range(n_f)] for p in range(n_v)]


def tally_skip_null(x_col, v_col, missing_aware: bool = True):
    """The operator used for B_{j,xi}: the 2-way tally with null entries of X
    discarded (and, with ``missing_aware``, missing entries of V as well)."""
    t = np.zeros((2, 2), dtype=np.int64)
    for ex, cv in zip(x_col, v_col):
        ev = allele_pair(cv)
        if ex == NULL:
            continue
        if missing_aware and ev == MISSING:
            continue
        if not missing_aware:
            ev = _canon(ev)
        for y in ex:
            for z in ev:
                t[y, z] += 1
    return t


def tally3_via_x(codes: np.ndarray, missing_aware: bool = True) -> np.ndarray:
    """[T, 8] tables for all i<j<k rebuilt from B_{j,xi} = X_{j,xi}^T o V by
    the mapping identities: entries with a = 0 take 2 B_{j,1} + B_{j,2},
    entries with a = 1 take 2 B_{j,3} + B_{j,2}."""
    n = codes.shape[0]
    out = np.zeros((n, n, n, 2, 2, 2), dtype=np.int64)
    for j in range(n):
        xs = {xi: x_matrix(codes, j, xi, missing_aware) for xi in (1, 2, 3)}
        for i in range(n):
            for k in range(n):
                b = {xi: tally_skip_null(xs[xi][i], codes[k], missing_aware) for xi in (1, 2, 3)}
                for bb in range(2):
                    for c in range(2):
                        out[i, j, k, 0, bb, c] = 2 * b[1][bb, c] + b[2][bb, c]
                        out[i, j, k, 1, bb, c] = 2 * b[3][bb, c] + b[2][bb, c]
    res = [out[i, j, k].reshape(8) for i in range(n) for j in range(i + 1, n)
           for k in range(j + 1, n)]
    return np.array(res, dtype=np.int64).reshape(-1, 8)


# ---------------------------------------------------------------------------
# Multi-allelic 2-way tallies (the s-state extension of Sec. 7, item 2).
# ---------------------------------------------------------------------------

def multi_tally2(a1_i, a2_i, a1_j, a2_j, s):
    """s x s table [a][b] for two vectors given as explicit allele pairs
    (a1[q], a2[q]), -1 in either marking a missing entry: every allele of one
    entry is paired with every allele of the other and the pair of states is
    tallied, as in the 2-way worked example of Sec. 2.1."""
    t = np.zeros((s, s), dtype=np.int64)
    for x1, x2, y1, y2 in zip(a1_i, a2_i, a1_j, a2_j):
        if min(x1, x2, y1, y2) < 0:
            continue
        for x in (x1, x2):
            for y in (y1, y2):
                t[x, y] += 1
    return t


def multi_all_pairs(a1, a2, s):
    """[P, s*s] tables for all i<j in lexicographic order, entry a*s + b."""
    n = a1.shape[0]
    out = [multi_tally2(a1[i], a2[i], a1[j], a2[j], s).reshape(s * s)
           for i in range(n) for j in range(i + 1, n)]
    return np.array(out, dtype=np.int64).reshape(-1, s * s)

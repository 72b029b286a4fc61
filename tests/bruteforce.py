"""Independent pure-Python brute force of the search, for tiny inputs only.

Written separately from oracle.c to pin it: its own digestion (substring
enumeration with the trypsin rule), its own residue masses (the integer
table in tests/golden, itself pinned to elemental formulas), no precursor-window index and no peak
table -- every (peak, fragment charge, ion) triple is compared directly -- and
the statistics through numpy/scipy library routines (Savitzky-Golay filter,
cumulative sums, least-squares polyfit).
"""
from __future__ import annotations

import math
import os
from fractions import Fraction
from itertools import combinations

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _elements():
    el = {}
    for line in open(os.path.join(GOLDEN, "elements.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        el[k] = float(v)
    return el


def residue_masses_da() -> dict:
    el = _elements()
    res = {}
    for line in open(os.path.join(GOLDEN, "residue_formulas.txt")):
        if line.startswith("#") or not line.strip():
            continue
        a, c, h, n, o, s = line.split()
        res[a] = int(c) * el["C"] + int(h) * el["H"] + int(n) * el["N"] + int(o) * el["O"] + int(s) * el["S"]
    return res


def _uda_table():
    t = {}
    for line in open(os.path.join(GOLDEN, "residue_uda.txt")):
        if line.startswith("#") or not line.strip():
            continue
        k, v = line.split()
        t[k] = int(v)
    return t


EL = _elements()
_UDA = _uda_table()
RES_UDA = {k: v for k, v in _UDA.items() if len(k) == 1}
WATER_UDA = _UDA["water"]
PROTON_UDA = _UDA["proton"]
# neutral losses and gains of the other ion series, from the elements
CO_UDA = round((EL["C"] + EL["O"]) * 1e6)
NH3_UDA = round((EL["N"] + 3 * EL["H"]) * 1e6)
H2_UDA = round(2 * EL["H"] * 1e6)
ION_SHIFT = {"a": -CO_UDA, "b": 0, "c": NH3_UDA, "x": CO_UDA - H2_UDA, "y": 0, "z": -NH3_UDA}


def is_cleavage_boundary(seq: str, pos: int) -> bool:
    """True when a peptide may start/end at `pos` (between seq[pos-1] and seq[pos])."""
    if pos == 0 or pos == len(seq):
        return True
    return seq[pos - 1] in "KR" and seq[pos] != "P"


def digest(seq: str, missed: int, min_len: int, max_len: int):
    """All substrings [s, e) bounded by cleavage boundaries, with at most
    `missed` boundaries strictly inside and length in range."""
    out = []
    for s in range(len(seq)):
        for e in range(s + 1, len(seq) + 1):
            if not (is_cleavage_boundary(seq, s) and is_cleavage_boundary(seq, e)):
                continue
            inside = sum(1 for p in range(s + 1, e) if is_cleavage_boundary(seq, p))
            if inside <= missed and min_len <= e - s <= max_len:
                out.append((s, e - s))
    return out


def sites_of(seq: str, start: int, length: int, mods):
    """[(position, delta)] in mask-bit order: N-terminus site first, then residues."""
    sites = []
    if start == 0:
        for m in mods:
            if m.nterm:
                sites.append((0, m.delta_uda))
                break
    for j in range(length):
        for m in mods:
            if not m.nterm and seq[start + j] in m.residues:
                sites.append((j, m.delta_uda))
                break
    return sites


def database(proteins: list[str], missed, min_len, max_len, mods, max_mods):
    """Sorted list of (mass, prot, start, len, mask, residue_masses)."""
    rows = []
    for p, seq in enumerate(proteins):
        for s, ln in digest(seq, missed, min_len, max_len):
            sites = sites_of(seq, s, ln, mods)
            for k in range(0, min(max_mods, len(sites)) + 1):
                for combo in combinations(range(len(sites)), k):
                    r = [RES_UDA[c] for c in seq[s:s + ln]]
                    mask = 0
                    for i in combo:
                        r[sites[i][0]] += sites[i][1]
                        mask |= 1 << i
                    rows.append((sum(r) + WATER_UDA, p, s, ln, mask, r))
    rows.sort(key=lambda t: t[:5])
    return rows


def round_half_away(x: float) -> int:
    f = Fraction(x)
    return math.floor(f + Fraction(1, 2)) if f >= 0 else -math.floor(-f + Fraction(1, 2))


def bin_of(m: int) -> int:
    return (m + 5000) // 10000


def hyperscore(nb: int, ny: int, s: int) -> float:
    return math.log10(math.factorial(nb) * math.factorial(ny) * s)


def evalue_numpy(hist: np.ndarray, top_h: float, n_scored: int):
    from scipy.signal import savgol_coeffs
    if n_scored == 0:
        return 1, float("nan")
    # the 5-point quadratic Savitzky-Golay window from scipy, applied as an exact
    # integer convolution (so equal smoothed values stay equal when the mode is taken)
    kern = np.rint(savgol_coeffs(5, 2) * 35.0).astype(np.int64)
    num = np.convolve(hist.astype(np.int64), kern, mode="same")
    hs = np.where(num < 0, 0, num) / 35.0
    total = hs.sum()
    mode = int(np.argmax(hs))
    last = min(511, int(math.floor(10.0 * top_h))) - 1
    tail = np.cumsum(hs[::-1])[::-1]
    xs, ys = [], []
    for j in range(mode, last + 1):
        sv = tail[j] / total if total > 0 else 0.0
        if sv > 0:
            xs.append(0.1 * j)
            ys.append(math.log10(sv))
    if len(xs) < 3:
        return 2, float("nan")
    w, b = np.polyfit(np.array(xs), np.array(ys), 1)
    if not w < 0:
        return 3, float("nan")
    return 0, n_scored * 10.0 ** (w * top_h + b)


def _q_sqrt(v, imax):
    """round(100 * sqrt(v / imax)) half up, in 50-digit decimal arithmetic."""
    from decimal import ROUND_FLOOR, Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        x = (Decimal(v) / Decimal(imax)).sqrt() * 100 + Decimal("0.5")
        return int(x.to_integral_value(rounding=ROUND_FLOOR))


def search(db_rows, mz, inten, prec_mz, z, window_is_ppm, window, T, top_b, top_k, kmin, noise_permille=0,
           intensity="linear", ions="by"):
    """One spectrum.  Returns dict with window, scored set, top hits, hist, e-value.
    noise_permille: peaks below that many thousandths of the most intense one are
    dropped before the top-B selection; intensity "sqrt": q from the square root
    of the relative intensity."""
    from fractions import Fraction
    n = len(mz)
    imax = max((float(v) for v in inten), default=0.0)
    alive = [i for i in range(n) if Fraction(float(inten[i])) * 1000 >= Fraction(imax) * noise_permille]
    order = sorted(alive, key=lambda i: (-float(inten[i]), float(mz[i]), i))[:top_b]
    peaks = []
    for i in order:
        if imax > 0:
            if intensity == "sqrt":
                t = _q_sqrt(float(inten[i]), imax)
            else:
                t = math.floor(float(inten[i]) / imax * 100.0 + 0.5)
            q = min(100, max(1, t))
        else:
            q = 1
        peaks.append((round_half_away(float(mz[i]) * 1e6), q))
    mq = z * (round_half_away(float(prec_mz) * 1e6) - PROTON_UDA)
    dm = (mq * window) // 1_000_000 if window_is_ppm else window
    cmax = max(1, z - 1)
    window_ids = [i for i, row in enumerate(db_rows) if abs(row[0] - mq) <= dm]
    scored = {}
    pairs_total = 0
    for pid in window_ids:
        r = db_rows[pid][5]
        L = len(r)
        bs = [sum(r[:i]) + PROTON_UDA + ION_SHIFT[t] for t in ions if t in "abc" for i in range(1, L)]
        ys = [sum(r[L - i:]) + WATER_UDA + PROTON_UDA + ION_SHIFT[t] for t in ions if t in "xyz" for i in range(1, L)]
        nb = ny = s = 0
        for (pm, q) in peaks:
            for c in range(1, cmax + 1):
                m1 = c * pm - (c - 1) * PROTON_UDA
                if m1 < 0:
                    continue
                pb = bin_of(m1)
                for ion in bs:
                    if abs(pb - bin_of(ion)) <= T:
                        nb += 1
                        s += q
                for ion in ys:
                    if abs(pb - bin_of(ion)) <= T:
                        ny += 1
                        s += q
        pairs_total += nb + ny
        if nb + ny >= kmin:
            scored[pid] = (nb, ny, s, hyperscore(nb, ny, s))
    ranked = sorted(scored.items(), key=lambda kv: (-kv[1][3], kv[0]))[:top_k]
    hist = np.zeros(512, dtype=np.int64)
    for (nb, ny, s, h) in scored.values():
        hist[min(511, int(math.floor(10.0 * h)))] += 1
    top_h = ranked[0][1][3] if ranked else 0.0
    st, ev = evalue_numpy(hist, top_h, len(scored))
    return {
        "lo": window_ids[0] if window_ids else 0,
        "hi": window_ids[-1] + 1 if window_ids else 0,
        "n_window": len(window_ids),
        "scored": scored,
        "top": ranked,
        "hist": hist,
        "status": st,
        "evalue": ev,
        "pairs_total": pairs_total,
    }

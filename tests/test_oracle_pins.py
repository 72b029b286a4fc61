"""Pins of the CPU oracle against things other than itself (no GPU needed).

Each test ties one part of the oracle to the paper, to chemistry, to a
closed form, to an independent library routine, or to the pure-Python brute
force in tests/bruteforce.py.
"""
import math
import os
from itertools import combinations

import numpy as np
import pytest

import oracle
from oracle import ModSpec
from paper_2102_02286_amd import synth
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _db(proteins, missed=2, min_len=2, max_len=40, mods=(), max_mods=0):
    res = np.frombuffer("".join(proteins).encode(), dtype=np.uint8)
    off = np.zeros(len(proteins) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in proteins])
    return oracle.Database(res, off, missed, min_len, max_len, list(mods), max_mods)


def _spectra(peak_lists, prec, charges):
    off = np.zeros(len(peak_lists) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in peak_lists])
    mz = np.array([m for pl in peak_lists for (m, _) in pl], np.float32)
    it = np.array([i for pl in peak_lists for (_, i) in pl], np.float32)
    return synth.Spectra(off, mz, it, np.asarray(prec, np.float64), np.asarray(charges, np.int8))


# --------------------------------------------------------------------------
# Masses: chemistry pins.
# --------------------------------------------------------------------------

def test_residue_masses_match_elemental_formulas():
    """Each oracle residue mass equals its elemental formula (AME 2016 atomic masses)."""
    letters = "GASPVTCLINDQKEMHFRYW"
    # one protein holding every residue, digested with enough missed cleavages to
    # produce the full-length peptide
    seq = "GASPVTCLINDQKEMHFRYW"
    db = _db([seq], missed=3, min_len=2, max_len=40)
    tab = db.table()
    full = [i for i in range(len(db)) if tab[i]["start"] == 0 and tab[i]["len"] == len(seq)]
    assert len(full) == 1
    r = db.residue_masses(full[0])
    expect = bf.residue_masses_da()
    for j, c in enumerate(letters):
        assert abs(r[j] - expect[c] * 1e6) <= 1.0, c


def test_golden_integer_masses_match_elemental_formulas():
    d = bf.residue_masses_da()
    for c, v in bf.RES_UDA.items():
        assert abs(v - d[c] * 1e6) <= 1.0, c
    assert abs(bf.WATER_UDA - (2 * bf.EL["H"] + bf.EL["O"]) * 1e6) <= 0.5
    assert abs(bf.PROTON_UDA - bf.EL["proton"] * 1e6) <= 0.5


def test_calibrant_peptide_masses():
    """[M+H]+ of standard calibration peptides, to the printed 4 decimals."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "calibrant_peptides.txt")) if not l.startswith("#")]
    for name, seq, mh in rows:
        db = _db([seq], missed=10, min_len=2, max_len=60)
        tab = db.table()
        full = [i for i in range(len(db)) if tab[i]["start"] == 0 and tab[i]["len"] == len(seq)]
        assert len(full) == 1, name
        m = tab[full[0]]["mass"]
        assert abs((m + bf.PROTON_UDA) * 1e-6 - float(mh)) <= 2e-4, name


def test_modification_deltas_match_elemental_formulas():
    el = bf.EL
    expect = {
        "Oxidation": el["O"],
        "Phospho": el["H"] + el["P"] + 3 * el["O"],
        "Acetyl": 2 * el["C"] + 2 * el["H"] + el["O"],
        "Deamidation": el["O"] - el["N"] - el["H"],
    }
    for m in (synth.OXIDATION, synth.PHOSPHO, synth.ACETYL_NTERM, synth.DEAMIDATION):
        uda = oracle.mods_from_synth([m])[0].delta_uda
        assert abs(uda - expect[m.name] * 1e6) <= 1.0, m.name


# --------------------------------------------------------------------------
# Ion series: closed form and the paper's worked example.
# --------------------------------------------------------------------------

def test_b_plus_y_equals_precursor_plus_two_protons():
    """b_i + y_(n-i) = M + 2 H+ exactly in integer uDa, with modifications."""
    prot = synth.make_proteome(30, seed=5)
    mods = oracle.mods_from_synth([synth.OXIDATION, synth.PHOSPHO, synth.ACETYL_NTERM])
    db = oracle.Database(prot.residues, prot.offsets, 1, 7, 30, mods, 2)
    rng = np.random.default_rng(0)
    for pid in rng.integers(0, len(db), size=300):
        mass = db.get(int(pid))[0]
        r = db.residue_masses(int(pid))
        b, y = oracle.ions(r)
        n = len(r)
        assert int(r.sum()) + bf.WATER_UDA == mass
        for i in range(1, n):
            assert b[i - 1] + y[n - i - 1] == mass + 2 * bf.PROTON_UDA


def test_mod_distance_worked_example():
    """Supplementary Text 3: p = MEGSYIRK shares 3 b/y ions with q (E*, I*) and
    6 with r (S*, Y*); Mod Distance 2 - a/max(len) = 1.625 and 1.25.

    The shared-ion counts come out of the oracle's full search path: the
    noise-free theoretical spectrum of p searched at T = 0 against a database
    holding p's modified forms."""
    p = "MEGSYIRK"
    mods = [ModSpec("EI", 16_000_000), ModSpec("SY", 80_000_000)]
    db = _db([p], missed=1, min_len=8, max_len=8, mods=mods, max_mods=2)
    tab = db.table()
    b, y = oracle.ions(np.array([bf.RES_UDA[c] for c in p], np.int64))
    peaks = [(m * 1e-6, 10.0) for m in np.concatenate([b, y])]
    mass_p = int(sum(bf.RES_UDA[c] for c in p) + bf.WATER_UDA)
    sp = _spectra([peaks], [(mass_p + bf.PROTON_UDA) * 1e-6], [1])
    ids, nb, ny, sq = db.scored(sp, 0, False, 10**12, 0, 1000, min_shared=1)
    counts = {}
    for i, a, c in zip(ids, nb, ny):
        start, ln, mask = tab[i]["start"], tab[i]["len"], tab[i]["mask"]
        counts[int(mask)] = int(a) + int(c)
    # sites of MEGSYIRK in bit order: E(2)->bit0, S(4)->bit1, Y(5)->bit2, I(6)->bit3
    mask_q = (1 << 0) | (1 << 3)
    mask_r = (1 << 1) | (1 << 2)
    rows = [l.split() for l in open(os.path.join(GOLDEN, "mod_distance_example.txt"))
            if l.strip() and not l.startswith("#") and not l.startswith("peptide")]
    expect = {r[0]: (int(r[3]), float(r[5])) for r in rows}
    assert counts[mask_q] == expect["q"][0] == 3
    assert counts[mask_r] == expect["r"][0] == 6
    assert 2 - counts[mask_q] / len(p) == pytest.approx(expect["q"][1])
    assert 2 - counts[mask_r] / len(p) == pytest.approx(expect["r"][1])
    assert counts[0] == 2 * (len(p) - 1)       # p against itself: every b and y ion


# --------------------------------------------------------------------------
# Database generation: brute force and combinatorics.
# --------------------------------------------------------------------------

HAND_PROTEINS = ["MKPAKRPGGKKAAR", "AAAAKAAAAARPAAAAKPAAAAR", "GGGGGGGK", "KRKRKRPK",
                 "MSTYMNQKAAMSSRLLLLLLK", "PEPTIDEKMSTYR"]


@pytest.mark.parametrize("missed,min_len,max_len", [(0, 1 + 1, 40), (1, 2, 40), (2, 3, 10), (3, 5, 12)])
def test_digestion_matches_substring_bruteforce(missed, min_len, max_len):
    prot = synth.make_proteome(8, seed=11, len_lo=20, len_hi=60)
    proteins = HAND_PROTEINS + [p.decode() for p in prot.as_list()]
    db = _db(proteins, missed=missed, min_len=min_len, max_len=max_len)
    tab = db.table()
    got = sorted(set((int(r["prot"]), int(r["start"]), int(r["len"])) for r in tab))
    want = sorted((p, s, ln) for p, seq in enumerate(proteins) for s, ln in bf.digest(seq, missed, min_len, max_len))
    assert got == want
    assert len(tab) == len(want)           # no modifications: one entry per peptide


def test_variant_counts_are_binomial_sums():
    """Each peptide with s sites appears sum_{j<=m} C(s, j) times (D = zeta * 2^m model)."""
    proteins = HAND_PROTEINS + ["MSSTTYYMK", "STYSTYSTYSTYR"]
    mods = [ModSpec("M", 15_994_915), ModSpec("STY", 79_966_331), ModSpec("", 42_010_565, nterm=True)]
    for max_mods in (0, 1, 2, 3):
        db = _db(proteins, missed=1, min_len=2, max_len=30, mods=mods, max_mods=max_mods)
        tab = db.table()
        groups = {}
        for r in tab:
            groups.setdefault((int(r["prot"]), int(r["start"]), int(r["len"])), []).append(int(r["mask"]))
        for (p, s, ln), masks in groups.items():
            seq = proteins[p][s:s + ln]
            n_sites = sum(c in "MSTY" for c in seq) + (1 if s == 0 else 0)
            assert len(masks) == sum(math.comb(n_sites, j) for j in range(min(max_mods, n_sites) + 1))
            assert len(set(masks)) == len(masks)
            assert all(bin(m).count("1") <= max_mods for m in masks)


def test_database_matches_python_bruteforce_with_mods():
    proteins = ["MSTYMNQKAAMSSRLLLLLLK", "PEPTIDEKMSTYRNQ", "ACDEFGHIKLMNPQRSTVWY"]
    mods_o = [ModSpec("M", 15_994_915), ModSpec("STY", 79_966_331), ModSpec("", 42_010_565, nterm=True),
              ModSpec("NQ", 984_016)]
    db = _db(proteins, missed=2, min_len=3, max_len=20, mods=mods_o, max_mods=2)
    rows = bf.database(proteins, 2, 3, 20, mods_o, 2)
    tab = db.table()
    assert len(tab) == len(rows)
    for i, r in enumerate(rows):
        assert (int(tab[i]["mass"]), int(tab[i]["prot"]), int(tab[i]["start"]), int(tab[i]["len"]),
                int(tab[i]["mask"])) == r[:5]
        assert list(db.residue_masses(i)) == r[5]


# --------------------------------------------------------------------------
# Scoring and statistics: closed forms and independent library routines.
# --------------------------------------------------------------------------

def test_hyperscore_closed_form():
    assert oracle.hyperscore(2, 3, 100) == pytest.approx(3.0791812460476247, rel=1e-15, abs=0)
    rng = np.random.default_rng(3)
    for _ in range(300):
        nb, ny, s = int(rng.integers(0, 60)), int(rng.integers(0, 60)), int(rng.integers(1, 20000))
        assert oracle.hyperscore(nb, ny, s) == pytest.approx(bf.hyperscore(nb, ny, s), rel=1e-13)


def test_savitzky_golay_matches_scipy_and_keeps_quadratics():
    from scipy.signal import savgol_coeffs, savgol_filter
    assert np.allclose(savgol_coeffs(5, 2) * 35.0, [-3, 12, 17, 12, -3])
    rng = np.random.default_rng(4)
    for _ in range(50):
        h = rng.integers(0, 1000, size=512).astype(np.int32)
        h[rng.random(512) < 0.3] = 0
        want = savgol_filter(h.astype(np.float64), 5, 2, mode="constant", cval=0.0)
        want = np.where(want < 0, 0.0, want)
        assert np.allclose(oracle.sg_smooth(h), want, rtol=1e-12, atol=1e-9)
    j = np.arange(512, dtype=np.int64)
    quad = (3 * (j - 200) ** 2 + 7 * j + 11).astype(np.int32)
    sm = oracle.sg_smooth(quad)
    assert np.array_equal(sm[2:-2], quad[2:-2].astype(np.float64))


def test_evalue_matches_numpy_pipeline():
    rng = np.random.default_rng(5)
    checked = 0
    for _ in range(200):
        h = np.zeros(512, np.int32)
        n = int(rng.integers(5, 5000))
        scores = rng.gumbel(2.5, 0.4, size=n)
        top = float(scores.max() + rng.uniform(0, 3))
        for s in list(scores) + [top]:
            h[min(511, int(math.floor(10.0 * s)))] += 1
        st, ev, w, b, npts = oracle.evalue(h, top, n + 1)
        st2, ev2 = bf.evalue_numpy(h, top, n + 1)
        assert st == st2
        if st == 0:
            assert ev == pytest.approx(ev2, rel=1e-9)
            checked += 1
    assert checked > 100


def test_evalue_special_cases():
    h = np.zeros(512, np.int32)
    assert oracle.evalue(h, 0.0, 0)[0] == 1               # nothing scored
    h[40] = 1
    assert oracle.evalue(h, 4.05, 1)[0] == 2              # top bin is the mode: no tail points
    h = np.zeros(512, np.int32)
    h[10:20] = np.arange(1, 11)                            # rising histogram up to the top hit
    st = oracle.evalue(h, 1.95, int(h.sum()))[0]
    assert st in (2, 3)


def test_evalue_geometric_tail_recovers_decay_rate():
    """A histogram halving every bin has survival ~ 2^-j, so the fitted slope is
    log10(1/2) / 0.1 = -3.0103 per hyperscore unit (up to the clipped first
    bins), and the fit equals an independent least-squares fit of the same points."""
    h = np.array([2 ** (30 - j) if j <= 30 else 0 for j in range(512)], dtype=np.int64).astype(np.int32)
    top_h = 1.65                                  # bin 16 -> fit bins mode..15
    st, ev, w, b, npts = oracle.evalue(h, top_h, 1000)
    assert st == 0
    assert w == pytest.approx(math.log10(0.5) / 0.1, rel=0.03)
    kern = np.array([-3, 12, 17, 12, -3], np.int64)
    num = np.convolve(h.astype(np.int64), kern, mode="same")
    hs = np.where(num < 0, 0, num) / 35.0
    mode = int(np.argmax(hs))
    tail = np.cumsum(hs[::-1])[::-1] / hs.sum()
    xs = 0.1 * np.arange(mode, 16)
    wf, bf_ = np.polyfit(xs, np.log10(tail[mode:16]), 1)
    assert npts == len(xs)
    assert w == pytest.approx(wf, rel=1e-9) and b == pytest.approx(bf_, rel=1e-9)
    assert ev == pytest.approx(1000 * 10 ** (wf * top_h + bf_), rel=1e-9)


# --------------------------------------------------------------------------
# Search: brute force on tiny inputs, invariances, self-search.
# --------------------------------------------------------------------------

def _tiny_case(seed, mods, max_mods, z_choices=(1, 2, 3, 4), n_spec=12, noise_peaks=(3, 15)):
    rng = np.random.default_rng(seed)
    prot = synth.make_proteome(4, seed=seed, len_lo=30, len_hi=70)
    proteins = [p.decode() for p in prot.as_list()]
    rows = bf.database(proteins, 1, 4, 25, mods, max_mods)
    peak_lists, prec, charges = [], [], []
    for s in range(n_spec):
        z = int(rng.choice(z_choices))
        src = rows[int(rng.integers(0, len(rows)))]
        r = src[5]
        L = len(r)
        ions = [sum(r[:i]) + bf.PROTON_UDA for i in range(1, L)] + \
               [sum(r[L - i:]) + bf.WATER_UDA + bf.PROTON_UDA for i in range(1, L)]
        pl = [(float(m) * 1e-6 + rng.normal(0, 0.004), float(rng.lognormal())) for m in ions if rng.random() < 0.7]
        if z >= 3:
            pl += [((float(m) * 1e-6 + 1.007276) / 2, float(rng.lognormal())) for m in ions if rng.random() < 0.5]
        pl += [(float(rng.uniform(100, 2000)), float(rng.lognormal())) for _ in range(int(rng.integers(*noise_peaks)))]
        if s % 5 == 3 and pl:                    # exact duplicate peaks and intensity ties
            pl += [pl[0], (pl[1][0] + 0.001, pl[1][1])] if len(pl) > 1 else [pl[0]]
        if s % 7 == 6:
            pl = []                               # empty spectrum
        peak_lists.append(pl)
        prec.append((src[0] * 1e-6 + z * 1.007276) / z)
        charges.append(z)
    res = np.frombuffer("".join(proteins).encode(), dtype=np.uint8)
    off = np.zeros(len(proteins) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in proteins])
    db = oracle.Database(res, off, 1, 4, 25, list(mods), max_mods)
    return db, rows, _spectra(peak_lists, prec, charges)


_ION_BITS = {"a": 1, "b": 2, "c": 4, "x": 8, "y": 16, "z": 32}


@pytest.mark.parametrize("seed,window_is_ppm,window,T,top_b,kmin,noise,inten,ions", [
    (0, False, 300_000_000, 1, 100, 1, 0, "linear", "by"),
    (1, False, 50_000_000, 2, 20, 3, 0, "linear", "by"),
    (2, True, 20, 2, 100, 1, 0, "linear", "by"),
    (3, False, 10**12, 0, 7, 2, 0, "linear", "by"),
    (4, False, 300_000_000, 1, 100, 1, 150, "linear", "by"),     # noise clearing before top-B
    (5, False, 300_000_000, 1, 10, 1, 400, "sqrt", "by"),        # noise clearing, square-root intensities
    (6, False, 10**12, 2, 100, 2, 0, "sqrt", "by"),
    (7, False, 300_000_000, 1, 100, 1, 0, "linear", "abcxyz"),   # every ion series
    (8, False, 10**12, 0, 100, 1, 0, "linear", "cz"),            # c and z only
    (9, True, 50, 2, 60, 2, 100, "sqrt", "axy"),
])
def test_search_matches_python_bruteforce(seed, window_is_ppm, window, T, top_b, kmin, noise, inten, ions):
    mods = [ModSpec("M", 15_994_915), ModSpec("STY", 79_966_331), ModSpec("", 42_010_565, nterm=True)]
    db, rows, sp = _tiny_case(seed, mods, 2)
    assert len(db) == len(rows)
    top_k = 5
    imode = oracle.INTENSITY_SQRT if inten == "sqrt" else oracle.INTENSITY_LINEAR
    itypes = sum(_ION_BITS[c] for c in ions)
    hits, stats, hist = db.search(sp, window_is_ppm, window, T, top_b, top_k, kmin, threads=3,
                                  noise_permille=noise, intensity=imode, ion_types=itypes)
    for s in range(sp.n):
        a, b = int(sp.peak_off[s]), int(sp.peak_off[s + 1])
        want = bf.search(rows, sp.mz[a:b], sp.intensity[a:b], sp.precursor_mz[s], int(sp.charge[s]),
                         window_is_ppm, window, T, top_b, top_k, kmin, noise_permille=noise, intensity=inten,
                         ions=ions)
        st = stats[s]
        assert int(st["n_window"]) == want["n_window"]
        if want["n_window"]:
            assert (int(st["lo"]), int(st["hi"])) == (want["lo"], want["hi"])
        assert int(st["n_scored"]) == len(want["scored"])
        assert int(st["pairs_total"]) == want["pairs_total"]
        assert np.array_equal(hist[s].astype(np.int64), want["hist"])
        for j in range(top_k):
            h = hits[s, j]
            if j < len(want["top"]):
                pid, (nb, ny, sq, hh) = want["top"][j]
                assert (int(h["id"]), int(h["n_b"]), int(h["n_y"]), int(h["sum_q"])) == (pid, nb, ny, sq)
                assert float(h["hyperscore"]) == pytest.approx(hh, rel=1e-12)
            else:
                assert int(h["id"]) == 0xFFFFFFFF and h["hyperscore"] == -np.inf
        assert int(st["status"]) == want["status"]
        if want["status"] == 0:
            assert float(st["evalue"]) == pytest.approx(want["evalue"], rel=1e-9)
        # full scored set
        ids, nb, ny, sq = db.scored(sp, s, window_is_ppm, window, T, top_b, min_shared=kmin, noise_permille=noise,
                                    intensity=imode, ion_types=itypes)
        got = {int(i): (int(x), int(y), int(q)) for i, x, y, q in zip(ids, nb, ny, sq)}
        assert got == {k: v[:3] for k, v in want["scored"].items()}


def _same(a, b):
    """Bitwise equality of result arrays (NaN e-values compare equal)."""
    a, b = np.ascontiguousarray(a), np.ascontiguousarray(b)
    return a.dtype == b.dtype and a.shape == b.shape and a.tobytes() == b.tobytes()


def test_search_invariant_under_permutations_and_splits():
    w = synth.workload("tiny")
    prot = synth.make_proteome(120, seed=0)
    sp = w.spectra(prot, n=60, seed=9)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0)
    args = (True, 10, 2, 100, 5, 4)
    h0, s0, g0 = db.search(sp, *args, threads=4)
    rng = np.random.default_rng(1)
    # permute peaks within each spectrum
    mz, it = sp.mz.copy(), sp.intensity.copy()
    for s in range(sp.n):
        a, b = int(sp.peak_off[s]), int(sp.peak_off[s + 1])
        p = rng.permutation(b - a) + a
        mz[a:b], it[a:b] = sp.mz[p], sp.intensity[p]
    sp2 = synth.Spectra(sp.peak_off, mz, it, sp.precursor_mz, sp.charge)
    h1, s1, g1 = db.search(sp2, *args, threads=2)
    assert _same(h0, h1) and _same(s0, s1) and _same(g0, g1)
    # permute spectra within the batch
    perm = rng.permutation(sp.n)
    h2, s2, g2 = db.search(sp.subset(perm), *args, threads=1)
    assert _same(h0[perm], h2) and _same(s0[perm], s2) and _same(g0[perm], g2)
    # split the batch in two
    ha, sa, ga = db.search(sp.subset(np.arange(0, 25)), *args)
    hb, sb, gb = db.search(sp.subset(np.arange(25, sp.n)), *args)
    assert _same(np.concatenate([ha, hb]), h0) and _same(np.concatenate([sa, sb]), s0)


def _permute_proteins(prot, perm):
    """The proteome with its proteins in the order `perm`."""
    seqs = [prot.residues[int(prot.offsets[i]):int(prot.offsets[i + 1])] for i in range(len(prot.offsets) - 1)]
    res = np.concatenate([seqs[i] for i in perm]).astype(np.uint8)
    off = np.zeros(len(perm) + 1, np.uint64)
    off[1:] = np.cumsum([len(seqs[i]) for i in perm])
    return res, off


def _peptide_keys(table, residues, offsets):
    """A protein-order-free name for every entry: its residues, whether it
    starts its protein (where an N-terminal modification may sit), its sites."""
    keys = []
    for r in table:
        a = int(offsets[int(r["prot"])]) + int(r["start"])
        keys.append((bytes(residues[a:a + int(r["len"])]), int(r["start"]) == 0, int(r["mask"])))
    return keys


def test_search_invariant_under_protein_order():
    """Permuting the proteins renumbers the peptides (ids follow mass, then
    protein), but every spectrum keeps its window, its scored set (as peptides
    with their counts), its histogram, expect value and top hyperscores."""
    from collections import Counter
    w = synth.workload("tiny")
    prot = synth.make_proteome(120, seed=0)
    mods = oracle.mods_from_synth([synth.OXIDATION, synth.ACETYL_NTERM])
    sp = w.spectra(prot, n=30, seed=9)
    res2, off2 = _permute_proteins(prot, np.random.default_rng(3).permutation(len(prot.offsets) - 1))
    db1 = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, mods, 2)
    db2 = oracle.Database(res2, off2, w.missed, w.min_len, w.max_len, mods, 2)
    assert len(db1) == len(db2)
    args = (True, 10, 2, 100, 5, 2)
    h1, s1, g1 = db1.search(sp, *args, threads=4)
    h2, s2, g2 = db2.search(sp, *args, threads=4)
    assert _same(s1, s2) and _same(g1, g2)
    assert _same(h1["hyperscore"], h2["hyperscore"])
    k1 = _peptide_keys(db1.table(), prot.residues, prot.offsets)
    k2 = _peptide_keys(db2.table(), res2, off2)
    n_sets = 0
    for s in range(sp.n):
        a = db1.scored(sp, s, *args[:4], min_shared=2)
        b = db2.scored(sp, s, *args[:4], min_shared=2)
        ca = Counter((k1[int(i)], int(x), int(y), int(q)) for i, x, y, q in zip(*a))
        cb = Counter((k2[int(i)], int(x), int(y), int(q)) for i, x, y, q in zip(*b))
        assert ca == cb
        n_sets += len(ca) > 0
    assert n_sets >= 20


def test_self_search_finds_source_peptide():
    """A noise-free theoretical spectrum of p shares every b/y ion with p
    (pairs >= 2(n-1)), and p ranks first unless an isobaric twin with a lower id
    ties it.  T = 1 bin, because float32 m/z moves a peak by up to ~60 uDa and can
    cross a bin edge."""
    prot = synth.make_proteome(40, seed=21)
    mods = oracle.mods_from_synth([synth.OXIDATION])
    db = oracle.Database(prot.residues, prot.offsets, 1, 7, 25, mods, 1)
    rng = np.random.default_rng(2)
    pids = [int(x) for x in rng.integers(0, len(db), size=25)]
    peak_lists, prec = [], []
    for pid in pids:
        b, y = oracle.ions(db.residue_masses(pid))
        peak_lists.append([(float(m) * 1e-6, 1.0 + (i % 7)) for i, m in enumerate(np.concatenate([b, y]))])
        prec.append((db.get(pid)[0] + 2 * bf.PROTON_UDA) * 1e-6 / 2)
    sp = _spectra(peak_lists, prec, [2] * len(pids))
    hits, stats, _ = db.search(sp, False, 5_000_000, 1, 1000, 5, 1)
    for s, pid in enumerate(pids):
        n = db.get(pid)[3]
        ids, nb, ny, _ = db.scored(sp, s, False, 5_000_000, 1, 1000, min_shared=1)
        k = list(ids).index(pid)
        assert int(nb[k]) + int(ny[k]) >= 2 * (n - 1)
        top = hits[s, 0]
        if int(top["id"]) != pid:
            # only a lower-id candidate with an equal or better score may outrank p
            mine = [j for j in range(5) if int(hits[s, j]["id"]) == pid]
            assert int(top["id"]) < pid and (not mine or hits[s, mine[0]]["hyperscore"] == top["hyperscore"])


def test_oracle_rejects_invalid_inputs():
    db = _db(["PEPTIDEKAAR"], missed=1, min_len=3, max_len=20)
    good = _spectra([[(300.0, 1.0)]], [500.0], [2])
    with pytest.raises(ValueError):
        db.search(good, False, 1, 1, 10, 0, 1)          # top_k = 0
    with pytest.raises(ValueError):
        db.search(good, False, 1, 1, 10, 5, 0)          # k_min = 0
    bad = _spectra([[(float("nan"), 1.0)]], [500.0], [2])
    with pytest.raises(ValueError):
        db.search(bad, False, 1, 1, 10, 5, 1)
    bad = _spectra([[(300.0, 1.0)]], [500.0], [0])
    with pytest.raises(ValueError):
        db.search(bad, False, 1, 1, 10, 5, 1)
    with pytest.raises(ValueError):
        _db(["PEPTIDEXK"])                               # non-standard residue


@pytest.mark.parametrize("z", [1, 2, 3])
def test_window_edges_are_inclusive(z):
    """filter_1 keeps a candidate whose mass differs from the query's by exactly
    the tolerance, and drops one a micro-dalton further (absolute and ppm)."""
    db = _db(["PEPTIDEK"], missed=0, min_len=8, max_len=8)
    assert len(db) == 1
    pep = sum(bf.RES_UDA[c] for c in "PEPTIDEK") + bf.WATER_UDA
    peaks = [[(300.0, 1.0)]]

    def window_of(mq, ppm, w):
        # precursor m/z whose rounded micro-dalton value gives neutral mass mq at charge z
        assert mq % z == 0
        prec = (mq // z + bf.PROTON_UDA) / 1e6
        _, st, _ = db.search(_spectra(peaks, [prec], [z]), ppm, w, 1, 10, 1, 1)
        return int(st[0]["n_window"])

    # every residue of the query mass modulo z, so both edges are hit exactly for some dm
    edges = 0
    for dm in range(1000, 1000 + z):
        for mq in range(pep - dm - 2 * z - (pep - dm) % z, pep + dm + 2 * z, z):
            inside = abs(pep - mq) <= dm
            edges += abs(pep - mq) == dm
            assert window_of(mq, False, dm) == int(inside), (dm, mq)
    assert edges >= 2
    # ppm: the tolerance is floor(M_q * ppm / 1e6) micro-daltons
    ppm = 10
    t0 = pep * ppm // 1_000_000
    near = [m for c in (pep - t0, pep + t0) for m in range(c - 6 * z - c % z, c + 6 * z, z)]
    for mq in near:
        tol = mq * ppm // 1_000_000
        assert window_of(mq, True, ppm) == int(abs(pep - mq) <= tol), mq


# --------------------------------------------------------------------------
# Partitions and result assembly (Superstep 4; Supplementary Algorithm 4).
# --------------------------------------------------------------------------

@pytest.mark.parametrize("G", [1, 2, 3, 4])
def test_shards_are_round_robin_slices(G):
    prot = synth.make_proteome(30, seed=4)
    mods = oracle.mods_from_synth([synth.OXIDATION])
    db = oracle.Database(prot.residues, prot.offsets, 1, 6, 25, mods, 1)
    whole = db.table()
    parts = [db.shard(G, g).table() for g in range(G)]
    assert sum(len(p) for p in parts) == len(whole)
    for g, p in enumerate(parts):
        assert _same(p, whole[g::G])
    with pytest.raises(ValueError):
        db.shard(G, G)


def test_assembly_orders_ties_by_global_id_and_adds_counts():
    """Two hand-made partition results of one spectrum whose whole-database
    window is ids [1, 7): partition 0 holds the even ids (local 1..3), partition
    1 the odd ones (local 0..2).  The expected merge is written out by hand: ids
    map back as local * G + g, equal hyperscores order by the global id, and
    histograms and counts add bin by bin."""
    empty = (np.uint32(0xFFFFFFFF), 0, 0, 0, 0, -np.inf)
    h0 = np.array([[(1, 3, 4, 50, 0, 5.0), (2, 2, 2, 30, 0, 4.0), empty]], oracle.HIT_DTYPE)
    h1 = np.array([[(0, 4, 3, 60, 0, 5.0), (1, 1, 3, 20, 0, 4.0), (2, 1, 3, 10, 0, 3.0)]], oracle.HIT_DTYPE)
    s0 = np.zeros(1, oracle.STAT_DTYPE); s1 = np.zeros(1, oracle.STAT_DTYPE)
    s0["n_window"], s0["n_scored"], s0["lo"], s0["hi"], s0["pairs_total"] = 3, 2, 1, 4, 11
    s1["n_window"], s1["n_scored"], s1["lo"], s1["hi"], s1["pairs_total"] = 3, 3, 0, 3, 17
    g0 = np.zeros((1, oracle.HIST_BINS), np.int32); g1 = np.zeros((1, oracle.HIST_BINS), np.int32)
    g0[0, 40], g0[0, 50] = 1, 1
    g1[0, 30], g1[0, 40], g1[0, 50] = 1, 1, 1
    hits, stats, hist = oracle.assemble([h0, h1], [s0, s1], [g0, g1])
    # (5.0, global 1), (5.0, global 2), (4.0, global 3) beat (4.0, global 4) and (3.0, global 5)
    assert [int(x) for x in hits[0]["id"]] == [1, 2, 3]
    assert list(hits[0]["hyperscore"]) == [5.0, 5.0, 4.0]
    assert [int(x) for x in hits[0]["sum_q"]] == [60, 50, 20]
    assert int(stats[0]["n_window"]) == 6 and int(stats[0]["n_scored"]) == 5
    assert int(stats[0]["pairs_total"]) == 28
    assert (int(stats[0]["lo"]), int(stats[0]["hi"])) == (1, 7)
    assert int(hist[0, 30]) == 1 and int(hist[0, 40]) == 2 and int(hist[0, 50]) == 2
    assert int(hist.sum()) == 5
    # one partition with nothing scored anywhere: no hits, no expect value
    z = np.zeros(1, oracle.STAT_DTYPE)
    e = np.array([[empty] * 3], oracle.HIT_DTYPE)
    g = np.zeros((1, oracle.HIST_BINS), np.int32)
    hits, stats, _ = oracle.assemble([e, e], [z, z], [g, g])
    assert int(stats[0]["status"]) == 1 and np.isnan(stats[0]["evalue"])
    assert all(int(x) == 0xFFFFFFFF for x in hits[0]["id"])


@pytest.mark.parametrize("G", [1, 2, 3, 5])
def test_partitioned_search_assembles_to_the_whole_search(G):
    """A candidate's shared peaks, hyperscore and histogram bin depend on that
    candidate alone, and the partitions split the database into disjoint sets, so
    searching every partition and assembling must reproduce the whole-database
    search exactly: hits, counts, window ranges, histograms, fit and expect
    values (the correctness claim behind Superstep 4)."""
    w = synth.workload("tiny")
    prot = synth.make_proteome(150, seed=0)
    mods = oracle.mods_from_synth([synth.OXIDATION])
    sp = w.spectra(prot, n=40, seed=12)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, mods, 1)
    args = (False, 300_000_000, 2, 100, 6, 3)        # +-300 Da open window
    h, s, g = db.search(sp, *args, threads=4)
    assert (s["status"] == 0).sum() >= 30            # the fit runs for most spectra
    parts = [db.shard(G, i).search(sp, *args, threads=4) for i in range(G)]
    ha, sa, ga = oracle.assemble([p[0] for p in parts], [p[1] for p in parts], [p[2] for p in parts])
    assert _same(h, ha) and _same(s, sa) and _same(g, ga)


# --------------------------------------------------------------------------
# log-Weibull (Gumbel) fit (Superstep 4; Supplementary Algorithm 4).
# --------------------------------------------------------------------------

def _gumbel_hist(mu, beta, total):
    """Counts of `total` scores drawn exactly from Gumbel(mu, beta), binned as
    the search bins hyperscores: bin j = [0.1 j, 0.1 (j + 1)), the last bin open."""
    from scipy.stats import gumbel_r
    edges = 0.1 * np.arange(oracle.HIST_BINS + 1)
    cdf = gumbel_r.cdf(edges, loc=mu, scale=beta)
    cdf[-1] = 1.0
    return np.round(total * np.diff(cdf)).astype(np.int32)


def _kept(h):
    """The histogram restricted to the window the Sampling section keeps (the
    brute-force placement of _sample_bruteforce), zero elsewhere."""
    lo = _sample_bruteforce(h)
    k = np.zeros(oracle.HIST_BINS, np.int32)
    k[lo:lo + oracle.SAMPLE_BINS] = np.maximum(h[lo:lo + oracle.SAMPLE_BINS], 0)
    return k


@pytest.mark.parametrize("mu,beta", [(20.0, 0.5), (12.5, 0.4), (24.0, 0.5)])
def test_gumbel_fit_recovers_location_and_scale(mu, beta):
    """On a histogram of an exact Gumbel(mu, beta) whose samples all lie in the
    kept window the moment fit returns mu and beta up to binning (a few 1e-3),
    and the expect value is N times the Gumbel survival function of scipy at the
    fitted parameters."""
    from scipy.stats import gumbel_r
    h = _gumbel_hist(mu, beta, 10**8)
    assert np.array_equal(_kept(h), h)
    N = int(h.sum())
    top = mu + 6 * beta
    st, ev, m, b, npts = oracle.evalue_gumbel(h, top, N)
    assert st == 0 and npts > 30
    assert abs(m - mu) < 5e-3 and abs(b - beta) < 5e-3 * beta
    assert ev == pytest.approx(N * gumbel_r.sf(top, loc=m, scale=b), rel=1e-12)
    # far tail: the survival still carries full relative precision
    st, ev_far, _, _, _ = oracle.evalue_gumbel(h, mu + 40 * beta, N)
    assert ev_far == pytest.approx(N * gumbel_r.sf(mu + 40 * beta, loc=m, scale=b), rel=1e-12)


def test_gumbel_moments_equal_numpy_moments_of_the_smoothed_kept_histogram():
    """The fit is the moment fit of the (independently pinned) smoothed
    histogram of the kept window: compare with numpy moments over bin centres.
    Mass at bin 0 makes the zero padding and the clamping of the smoothing
    matter; a wide Gumbel loses its far tail to the window; and because the
    quadratic Savitzky-Golay window keeps the first two moments, the raw
    histogram of a smooth interior distribution gives the same answer."""
    k_gamma = 0.5772156649015329
    x = 0.1 * np.arange(oracle.HIST_BINS) + 0.05
    for h in [np.bincount([0, 0, 0, 1, 1, 5, 5, 9], minlength=oracle.HIST_BINS).astype(np.int32) * 10,
              _gumbel_hist(25.0, 3.0, 10**7), _gumbel_hist(20.0, 2.0, 10**7)]:
        hs = oracle.sg_smooth(_kept(h))
        m = np.sum(hs * x) / np.sum(hs)
        v = np.sum(hs * (x - m) ** 2) / np.sum(hs)
        beta = np.sqrt(6 * v) / np.pi
        st, ev, mu_f, beta_f, _ = oracle.evalue_gumbel(h, 3.0, 1000)
        assert st == 0
        assert mu_f == pytest.approx(m - k_gamma * beta, rel=1e-12) and beta_f == pytest.approx(beta, rel=1e-12)
    # interior (no mass near either end of the window): smoothing keeps the
    # moments of the raw histogram
    h = _gumbel_hist(20.0, 0.5, 10**7)
    m0 = np.sum(h * x) / h.sum()
    v0 = np.sum(h * (x - m0) ** 2) / h.sum()
    _, _, mu_f, beta_f, _ = oracle.evalue_gumbel(h, 30.0, int(h.sum()))
    # (up to the few sparse tail bins where smoothing goes negative and is clamped)
    assert beta_f == pytest.approx(np.sqrt(6 * v0) / np.pi, rel=2e-5)
    assert mu_f == pytest.approx(m0 - k_gamma * np.sqrt(6 * v0) / np.pi, rel=2e-5)


def test_gumbel_fit_sees_only_the_kept_samples():
    """Sampling section: the far tail a 256-byte record prunes is what the fitted
    distribution stands in for.  Counts added beyond the kept window leave the
    fit unchanged, and a record shifted back gives the full histogram's fit bit
    for bit whenever no count saturated and the shifted-back histogram places
    its window where the record's is (it does unless one of the three largest
    counts was pruned) -- on random histograms of every shape."""
    rng = np.random.default_rng(24)
    h = _gumbel_hist(20.0, 2.0, 10**6)
    lo = _sample_bruteforce(h)
    far = h.copy()
    far[lo + oracle.SAMPLE_BINS:] += 3                     # a longer tail past the window
    assert _sample_bruteforce(far) == lo
    a, b = oracle.evalue_gumbel(h, 30.0, 10**6), oracle.evalue_gumbel(far, 30.0, 10**6)
    assert a[0] == b[0] == 0 and a[1:4] == b[1:4]
    n_checked = 0
    for _ in range(300):
        h = np.zeros(oracle.HIST_BINS, np.int32)
        a0 = int(rng.integers(0, oracle.HIST_BINS))
        b0 = min(oracle.HIST_BINS, a0 + int(rng.integers(1, [30, 121, 300, 512][int(rng.integers(0, 4))])))
        h[a0:b0] = rng.integers(0, [3, 50, 1000, 80000][int(rng.integers(0, 4))], b0 - a0)
        n = int(h.sum())
        rec = oracle.sample(h, [n])
        if int(rec["flags"][0]) & 1:                       # a saturated count: the record differs
            continue
        back = oracle.unsample(rec)[0]
        if _sample_bruteforce(back) != int(rec["lo"][0]):
            continue
        full, samp = oracle.evalue_gumbel(h, 30.0, n), oracle.evalue_gumbel(back, 30.0, n)
        assert full[0] == samp[0]
        if full[0] == 0:
            assert full[1:4] == samp[1:4]
            n_checked += 1
    assert n_checked > 100


def test_gumbel_special_cases():
    h = np.zeros(oracle.HIST_BINS, np.int32)
    assert oracle.evalue_gumbel(h, 1.0, 0)[0] == 1                       # nothing scored
    h[0] = 5                                                             # smoothed: bins 0 and 1 only
    st, ev, _, _, npts = oracle.evalue_gumbel(h, 1.0, 5)
    assert st == 2 and npts == 2 and np.isnan(ev)
    h[0], h[100] = 0, 7                                                  # one bin spreads to three
    st, ev, mu, beta, npts = oracle.evalue_gumbel(h, 10.05, 7)
    assert st == 0 and npts == 3 and mu < 10.05 < mu + 3 * beta and 0 < ev < 7


def test_search_and_assembly_with_the_gumbel_fit():
    """The fit is chosen per search; both fits see the same histogram, and the
    partitioned search assembles to the whole one with either."""
    w = synth.workload("tiny")
    prot = synth.make_proteome(150, seed=0)
    sp = w.spectra(prot, n=30, seed=12)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, [], 0)
    args = (False, 300_000_000, 2, 100, 6, 3)
    ht, st, gt = db.search(sp, *args, threads=4)
    hg, sg, gg = db.search(sp, *args, threads=4, fit=oracle.FIT_GUMBEL)
    assert _same(ht, hg) and _same(gt, gg)
    ok = sg["status"] == 0
    assert ok.sum() >= 25
    for s in np.nonzero(ok)[0][:10]:
        want = oracle.evalue_gumbel(gg[s], ht[s, 0]["hyperscore"], int(st[s]["n_scored"]))[1]
        assert sg[s]["evalue"] == want
    parts = [db.shard(3, i).search(sp, *args, threads=4, fit=oracle.FIT_GUMBEL) for i in range(3)]
    ha, sa, ga = oracle.assemble([p[0] for p in parts], [p[1] for p in parts], [p[2] for p in parts],
                                 fit=oracle.FIT_GUMBEL)
    assert _same(hg, ha) and _same(sg, sa) and _same(gg, ga)


def test_preprocessing_special_cases():
    """Noise threshold 0 keeps every peak; a threshold of 1000 keeps only the
    most intense peak(s); square-root q of exact squares: I / Imax = (k/100)^2
    gives q = k, and the rounding edge (k - 1/2)^2 is rounded up."""
    db = _db(["MPEPTIDEKAAGLR"], missed=1, min_len=3, max_len=20)
    pep = db.residue_masses(0)
    b, y = oracle.ions(pep)
    mz = [float(m) * 1e-6 for m in np.concatenate([b, y])]
    prec = (db.get(0)[0] + 2 * bf.PROTON_UDA) * 1e-6 / 2
    ints = [1.0 + i for i in range(len(mz))]
    sp = _spectra([list(zip(mz, ints))], [prec], [2])
    full = db.search(sp, False, 10**9, 0, 100, 5, 1)
    zero = db.search(sp, False, 10**9, 0, 100, 5, 1, noise_permille=0)
    assert _same(full[0], zero[0]) and _same(full[1], zero[1])
    top = db.search(sp, False, 10**9, 0, 100, 5, 1, noise_permille=1000)
    pairs = int(top[1][0]["pairs_total"])
    assert 0 < pairs < int(full[1][0]["pairs_total"])
    # square-root intensities: only the intensity sums change
    imax = 10000.0
    for k in [1, 7, 50, 99, 100]:
        v = imax * (k / 100.0) ** 2
        assert bf._q_sqrt(v, imax) == k
    edge = imax * (6.5 / 100.0) ** 2                 # sqrt = 0.065 exactly: rounds half up to 7
    assert bf._q_sqrt(edge, imax) == 7
    # (exact ties like this one are decided on the fp64 value 10^4 * I / Imax, so the
    # spectrum below stays off them)
    sp2 = _spectra([[(mz[0], imax), (mz[1], imax * 0.00423), (mz[2], imax * 0.0049)]], [prec], [2])
    ids, nb, ny, sq = db.scored(sp2, 0, False, 10**9, 0, 100, min_shared=1, intensity=oracle.INTENSITY_SQRT)
    k = list(ids).index(0)
    assert int(sq[k]) == 100 + 7 + 7                  # sqrt(0.00423) = 0.06504, sqrt(0.0049) = 0.07
    ids, nb, ny, sq = db.scored(sp2, 0, False, 10**9, 0, 100, min_shared=1)
    assert int(sq[list(ids).index(0)]) == 100 + 1 + 1  # linear: 0.423 and 0.49 both round to 0, clamped to 1


def test_other_ion_series_closed_forms():
    """From the element masses: c_i + z_(n-i) = M + 2 H+ and a_i + x_(n-i) =
    M + 2 H+ - H2; a single peak placed on each series' first ion of a peptide
    matches it through the oracle only when that series is switched on."""
    assert bf.CO_UDA == 27994915 and bf.NH3_UDA == 17026549 and bf.H2_UDA == 2015650
    db = _db(["MPEPTIDEKAAGLR"], missed=1, min_len=3, max_len=20)
    pid = 0
    r = [int(x) for x in db.residue_masses(pid)]
    M, n = db.get(pid)[0], len(r)
    for i in range(1, n):
        pre, suf = sum(r[:i]), sum(r[i:])
        c = pre + bf.PROTON_UDA + bf.NH3_UDA
        z = suf + bf.WATER_UDA + bf.PROTON_UDA - bf.NH3_UDA
        a = pre + bf.PROTON_UDA - bf.CO_UDA
        x = suf + bf.WATER_UDA + bf.PROTON_UDA + bf.CO_UDA - bf.H2_UDA
        assert c + z == M + 2 * bf.PROTON_UDA
        assert a + x == M + 2 * bf.PROTON_UDA - bf.H2_UDA
    prec = (M + 2 * bf.PROTON_UDA) * 1e-6 / 2
    firsts = {"a": r[0] + bf.PROTON_UDA - bf.CO_UDA, "c": r[0] + bf.PROTON_UDA + bf.NH3_UDA,
              "x": r[-1] + bf.WATER_UDA + bf.PROTON_UDA + bf.CO_UDA - bf.H2_UDA,
              "z": r[-1] + bf.WATER_UDA + bf.PROTON_UDA - bf.NH3_UDA}
    for t, m in firsts.items():
        sp = _spectra([[(m * 1e-6, 1.0)]], [prec], [2])
        ids, nb, ny, sq = db.scored(sp, 0, False, 10**9, 0, 10, min_shared=1, ion_types=_ION_BITS[t])
        got = dict(zip(ids.tolist(), zip(nb.tolist(), ny.tolist())))
        # N-terminal series count in n_b, C-terminal ones in n_y
        assert pid in got and (got[pid][0] if t in "ac" else got[pid][1]) >= 1
        assert (got[pid][1] if t in "ac" else got[pid][0]) == 0


def test_ion_series_offsets_at_bin_edges():
    """Modification shifts chosen so that the doubly modified GAK has its c1 ion
    at 4999 and its z1 ion at 5000 uDa past a multiple of 10000, the two sides
    of a bin edge: a 1-uDa error in NH3 (or CO) moves them to the other bin, and
    with T = 0 a peak at the centre of the right bin then no longer matches."""
    mods = [ModSpec("", 42_009_710, nterm=True), ModSpec("K", 15_998_745)]
    db = _db(["GAK"], missed=0, min_len=3, max_len=3, mods=mods, max_mods=2)
    tab = db.table()
    pid = int(np.nonzero(tab["mask"] == 3)[0][0])
    r = [int(x) for x in db.residue_masses(pid)]
    c1 = r[0] + bf.PROTON_UDA + bf.NH3_UDA
    z1 = r[-1] + bf.WATER_UDA + bf.PROTON_UDA - bf.NH3_UDA
    assert c1 % 10000 == 4999 and z1 % 10000 == 5000
    peaks = [(bf.bin_of(c1) * 0.01, 1.0), (bf.bin_of(z1) * 0.01, 1.0)]
    prec = (int(tab["mass"][pid]) + 2 * bf.PROTON_UDA) * 1e-6 / 2
    sp = _spectra([peaks], [prec], [2])
    ids, nb, ny, sq = db.scored(sp, 0, False, 10**9, 0, 10, min_shared=1, ion_types=4 | 32)
    k = list(ids).index(pid)
    assert (int(nb[k]), int(ny[k])) == (1, 1)
    want = bf.search([(int(t["mass"]), 0, 0, 0, 0, db.residue_masses(i).tolist()) for i, t in enumerate(tab)],
                     sp.mz, sp.intensity, prec, 2, False, 10**9, 0, 10, 5, 1, ions="cz")
    assert want["scored"][pid][:2] == (1, 1)


# --------------------------------------------------------------------------
# Sampled intermediate results (Sampling section and its figure; the shift of
# Superstep 4's "addition and shift").
# --------------------------------------------------------------------------

def _sample_bruteforce(h):
    """The reading written as a search: the mean from the three most intense
    nonzero bins (sorted by count desc, bin asc), then the first window
    placement that starts no earlier than the head and no more than 60 bins
    below the mean; placements end at bin 511."""
    nz = [j for j in range(oracle.HIST_BINS) if h[j] > 0]
    if not nz:
        return 0
    top = sorted(nz, key=lambda j: (-int(h[j]), j))[:3]
    mean = sum(top) // len(top)
    for lo in range(0, oracle.HIST_BINS - oracle.SAMPLE_BINS + 1):
        if lo >= nz[0] and lo >= mean - oracle.SAMPLE_HEAD:
            return lo
    return oracle.HIST_BINS - oracle.SAMPLE_BINS


def _hand_hist(pairs, n=oracle.HIST_BINS):
    h = np.zeros(n, np.int32)
    for j, v in pairs:
        h[j] = v
    return h


def test_sampling_hand_worked_cases():
    """Cases worked out by hand from the reading (window of 120 bins; mean =
    floor of the average bin of the three largest counts)."""
    # narrow distribution: everything fits, the window starts at the head
    h = _hand_hist([(j, 5) for j in range(20, 40)] + [(30, 100), (31, 90), (35, 80)])
    r = oracle.sample(h[None], [7])[0]
    assert int(r["lo"]) == 20 and int(r["flags"]) == 0 and int(r["n_scored"]) == 7
    assert np.array_equal(oracle.unsample(r[None])[0], h)
    # long head: mean (150 + 151 + 152) / 3 = 151, window [91, 211): bins 0..90 are cut
    h = _hand_hist([(j, 1) for j in range(0, 201)] + [(150, 1000), (151, 900), (152, 800)])
    r = oracle.sample(h[None], [0])[0]
    assert int(r["lo"]) == 91 and int(r["flags"]) == 2
    u = oracle.unsample(r[None])[0]
    assert u[:91].sum() == 0 and np.array_equal(u[91:201], h[91:201]) and u[201:].sum() == 0
    # four equal counts: the three lowest bins are the most intense, mean 200, window [140, 260)
    h = _hand_hist([(100, 10), (200, 10), (300, 10), (400, 10)])
    r = oracle.sample(h[None], [40])[0]
    assert int(r["lo"]) == 140 and int(r["flags"]) == 2
    assert oracle.unsample(r[None])[0].sum() == 10
    # distribution against the top of the range: the window ends at bin 511
    h = _hand_hist([(j, 3) for j in range(450, 512)])
    r = oracle.sample(h[None], [186])[0]
    assert int(r["lo"]) == 392 and int(r["flags"]) == 0
    assert np.array_equal(oracle.unsample(r[None])[0], h)
    # saturation of a 16-bit sample
    h = _hand_hist([(5, 70000), (6, 3)])
    r = oracle.sample(h[None], [70003])[0]
    assert int(r["lo"]) == 5 and int(r["count"][0]) == 65535 and int(r["count"][1]) == 3
    assert int(r["flags"]) == 1
    # empty distribution
    r = oracle.sample(np.zeros((1, oracle.HIST_BINS), np.int32), [0])[0]
    assert int(r["lo"]) == 0 and int(r["flags"]) == 0 and int(r["count"].sum()) == 0


def test_sampling_matches_bruteforce_and_loses_only_outside_the_window():
    """Random histograms of every shape (narrow, wide, long heads, long tails,
    ties, edges): the window matches the brute-force search, kept counts equal
    the histogram inside it (saturated), and the flags say exactly whether
    anything was lost."""
    rng = np.random.default_rng(5)
    hs = []
    for _ in range(400):
        h = np.zeros(oracle.HIST_BINS, np.int32)
        kind = rng.integers(0, 4)
        a = int(rng.integers(0, oracle.HIST_BINS))
        b = min(oracle.HIST_BINS, a + int(rng.integers(1, [30, 121, 300, 512][kind])))
        h[a:b] = rng.integers(0, [3, 50, 1000, 80000][int(rng.integers(0, 4))], b - a)
        if rng.random() < 0.3:                      # ties among the largest counts
            h[rng.integers(a, b, 3)] = h.max()
        hs.append(h)
    hs = np.stack(hs)
    recs = oracle.sample(hs, np.arange(len(hs)))
    back = oracle.unsample(recs)
    for h, r, u in zip(hs, recs, back):
        lo = _sample_bruteforce(h)
        assert int(r["lo"]) == lo
        w = slice(lo, lo + oracle.SAMPLE_BINS)
        assert np.array_equal(u[w], np.minimum(h[w], 65535))
        assert u.sum() == np.minimum(h[w], 65535).sum()
        assert bool(r["flags"] & 1) == bool((h[w] > 65535).any())
        outside = h.copy()
        outside[w] = 0
        assert bool(r["flags"] & 2) == bool((outside > 0).any())
    assert int(recs["n_scored"][17]) == 17


def test_sampled_assembly_equals_full_assembly_when_lossless():
    """Partition results sampled to 256 bytes, shifted back and added give the
    same assembled results as the full histograms whenever no sample was lost
    (the usual case: hyperscores of one spectrum span well under 12 units)."""
    w = synth.workload("tiny")
    prot = synth.make_proteome(150, seed=0)
    mods = oracle.mods_from_synth([synth.OXIDATION])
    sp = w.spectra(prot, n=40, seed=12)
    db = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len, mods, 1)
    args = (False, 300_000_000, 2, 100, 6, 3)
    G = 3
    parts = [db.shard(G, i).search(sp, *args, threads=4) for i in range(G)]
    recs = [oracle.sample(p[2], p[1]["n_scored"]) for p in parts]
    lossless = np.all([r["flags"] == 0 for r in recs], axis=0)
    assert lossless.sum() >= 20                      # a lone far-out top hit is the usual loss
    full = oracle.assemble([p[0] for p in parts], [p[1] for p in parts], [p[2] for p in parts])
    samp = oracle.assemble([p[0] for p in parts], [p[1] for p in parts], [oracle.unsample(r) for r in recs])
    assert _same(full[0], samp[0])                   # hits never depend on the histogram
    assert np.array_equal(full[1]["n_scored"], samp[1]["n_scored"])
    assert _same(full[1][lossless], samp[1][lossless]) and _same(full[2][lossless], samp[2][lossless])
    # where samples were lost, the assembled histogram is the full one cut to the windows
    for i in np.nonzero(~lossless)[0]:
        assert (samp[2][i] <= full[2][i]).all() and samp[2][i].sum() < full[2][i].sum()


def test_scores_past_51_1_land_in_the_open_last_bin():
    """A 40-residue peptide whose every b and y ion is a peak scores
    H = log10(39! 39! S) ~ 96, far past 51.1: it must be counted in the open
    last histogram bin 511 (not past the array), and the tail fit must stop at
    bin 510, the bin below the top hit's clamped bin.  Checked against the
    brute force, which clamps with min(511, floor(10 H)) on its own."""
    pep = "GASPVTCLINDQEMHFYWGASPVTCLINDQEMHFYWGAGK"          # no K/R inside, ends with K
    assert len(pep) == 40
    rng = np.random.default_rng(51)
    filler = "".join(rng.choice(list("GASPVTLINDQEMHFYWKR"), 300))
    proteins = [pep + "R" + filler[:150], filler[150:]]
    rows = bf.database(proteins, 1, 4, 45, [], 0)
    res = np.frombuffer("".join(proteins).encode(), dtype=np.uint8)
    off = np.zeros(len(proteins) + 1, np.uint64)
    off[1:] = np.cumsum([len(p) for p in proteins])
    db = oracle.Database(res, off, 1, 4, 45, [], 0)
    assert len(db) == len(rows) and len(rows) > 30
    src = [r for r in rows if r[1] == 0 and r[2] == 0 and r[3] == 40][0]
    r = src[5]
    ions = [sum(r[:i]) + bf.PROTON_UDA for i in range(1, 40)] + \
           [sum(r[40 - i:]) + bf.WATER_UDA + bf.PROTON_UDA for i in range(1, 40)]
    peaks = [(float(m) * 1e-6, 10.0) for m in ions]
    peaks += [(float(rng.uniform(100, 2000)), float(rng.lognormal())) for _ in range(40)]
    sp = _spectra([peaks], [(src[0] * 1e-6 + 2 * 1.007276) / 2], [2])
    for T, fit in ((0, oracle.FIT_TAIL), (1, oracle.FIT_TAIL), (1, oracle.FIT_GUMBEL)):
        hits, stats, hist = db.search(sp, False, 10**12, T, 200, 5, 1, threads=1, fit=fit)
        want = bf.search(rows, sp.mz, sp.intensity, sp.precursor_mz[0], 2, False, 10**12, T, 200, 5, 1)
        top = float(hits[0, 0]["hyperscore"])
        assert top > 51.1 and int(hits[0, 0]["n_b"]) >= 39 and int(hits[0, 0]["n_y"]) >= 39
        assert top == pytest.approx(want["top"][0][1][3], rel=1e-12)
        assert np.array_equal(hist[0].astype(np.int64), want["hist"])
        assert hist[0, 511] >= 1 and hist[0, 511] == sum(1 for v in want["scored"].values() if v[3] >= 51.1)
        if fit == oracle.FIT_TAIL:
            assert int(stats[0]["status"]) == want["status"]
            if want["status"] == 0:
                assert float(stats[0]["evalue"]) == pytest.approx(want["evalue"], rel=1e-9)
            # the fit ends at bin 510: a top hit anywhere in the open bin (51.15) fits the same
            # points, one in bin 510 (51.05) one point fewer
            ns = int(stats[0]["n_scored"])
            st1, ev1, w1, b1, n1 = oracle.evalue(hist[0], top, ns)
            assert st1 == int(stats[0]["status"]) == 0
            assert n1 == oracle.evalue(hist[0], 51.15, ns)[4] == oracle.evalue(hist[0], 51.05, ns)[4] + 1
            assert ev1 == pytest.approx(ns * 10.0 ** (w1 * top + b1), rel=1e-12)

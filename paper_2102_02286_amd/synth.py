"""Seeded synthetic inputs: proteomes, MS/MS spectra and request arrival streams.

This module only *makes data*.  It holds none of the search arithmetic: it does
not bin, window, count, score or fit anything, and both the CPU oracle and the
GPU library consume its arrays as plain inputs.  To make spectra that look like
the paper's workloads (tryptic peptides with variable modifications, b/y
fragments with m/z noise, uniform noise peaks, lognormal intensities), it
carries its own float64 residue-mass table and its own small tryptic digester.
Those values only shape the inputs; no expected result is ever taken from here.

Stand-in for the paper's PRIDE spectra and UniProt databases (Experimental
Setup section), which are not available: every workload here is synthetic.

RNG: numpy PCG64 ``default_rng``; proteome seed 0, spectra seed 1, arrival
stream seed 2, unless a caller overrides them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

AMINO = b"ACDEFGHIKLMNPQRSTVWY"

# float64 Da monoisotopic residue masses, used only to synthesise fragment m/z.
_RES_DA = {
    "G": 57.02146, "A": 71.03711, "S": 87.03203, "P": 97.05276, "V": 99.06841,
    "T": 101.04768, "C": 103.00919, "L": 113.08406, "I": 113.08406, "N": 114.04293,
    "D": 115.02694, "Q": 128.05858, "K": 128.09496, "E": 129.04259, "M": 131.04049,
    "H": 137.05891, "F": 147.06841, "R": 156.10111, "Y": 163.06333, "W": 186.07931,
}
_WATER_DA = 18.010565
_PROTON_DA = 1.007276

_RES_LUT = np.zeros(256, dtype=np.float64)
for _k, _v in _RES_DA.items():
    _RES_LUT[ord(_k)] = _v


@dataclass(frozen=True)
class Mod:
    """A variable modification: residues it may sit on, or the protein N-terminus."""
    name: str
    residues: str          # e.g. "STY"; ignored when nterm is True
    delta_da: float        # float Da, as a workload description prints it
    nterm: bool = False    # True: protein N-terminus only


OXIDATION = Mod("Oxidation", "M", 15.994915)
PHOSPHO = Mod("Phospho", "STY", 79.966331)
ACETYL_NTERM = Mod("Acetyl", "", 42.010565, nterm=True)
DEAMIDATION = Mod("Deamidation", "NQ", 0.984016)


@dataclass
class Proteome:
    residues: np.ndarray      # uint8, all proteins concatenated
    offsets: np.ndarray       # uint64 [n+1]

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def protein(self, i: int) -> bytes:
        return self.residues[self.offsets[i]:self.offsets[i + 1]].tobytes()

    def as_list(self) -> list[bytes]:
        return [self.protein(i) for i in range(self.n)]


@dataclass
class Spectra:
    """Host CSR batch of spectra (the boundary's input layout)."""
    peak_off: np.ndarray      # uint64 [n+1]
    mz: np.ndarray            # float32 [nnz]
    intensity: np.ndarray     # float32 [nnz]
    precursor_mz: np.ndarray  # float64 [n]
    charge: np.ndarray        # int8 [n]
    # provenance of each spectrum (generator bookkeeping, not an input)
    is_noise: np.ndarray = field(default=None)  # bool [n]

    @property
    def n(self) -> int:
        return int(self.peak_off.shape[0] - 1)

    def subset(self, idx) -> "Spectra":
        idx = np.asarray(idx, dtype=np.int64)
        lo = self.peak_off[idx].astype(np.int64)
        hi = self.peak_off[idx + 1].astype(np.int64)
        counts = hi - lo
        off = np.zeros(len(idx) + 1, dtype=np.uint64)
        np.cumsum(counts, out=off[1:])
        sel = np.concatenate([np.arange(a, b) for a, b in zip(lo, hi)]) if len(idx) else np.zeros(0, np.int64)
        sel = sel.astype(np.int64)
        return Spectra(off, self.mz[sel].copy(), self.intensity[sel].copy(),
                       self.precursor_mz[idx].copy(), self.charge[idx].copy(),
                       None if self.is_noise is None else self.is_noise[idx].copy())

    def slice(self, a: int, b: int) -> "Spectra":
        """Spectra [a, b) as a new batch (contiguous peaks, offsets rebased)."""
        p0, p1 = int(self.peak_off[a]), int(self.peak_off[b])
        return Spectra((self.peak_off[a:b + 1] - np.uint64(p0)).copy(), self.mz[p0:p1].copy(),
                       self.intensity[p0:p1].copy(), self.precursor_mz[a:b].copy(), self.charge[a:b].copy(),
                       None if self.is_noise is None else self.is_noise[a:b].copy())

    @staticmethod
    def concat(parts: list["Spectra"]) -> "Spectra":
        off = [np.zeros(1, np.uint64)]
        base = 0
        for p in parts:
            off.append(p.peak_off[1:] + np.uint64(base))
            base += int(p.peak_off[-1])
        noise = None
        if all(p.is_noise is not None for p in parts):
            noise = np.concatenate([p.is_noise for p in parts])
        return Spectra(np.concatenate(off), np.concatenate([p.mz for p in parts]),
                       np.concatenate([p.intensity for p in parts]),
                       np.concatenate([p.precursor_mz for p in parts]),
                       np.concatenate([p.charge for p in parts]), noise)


def make_proteome(n_proteins: int, seed: int = 0, len_lo: int = 100, len_hi: int = 600) -> Proteome:
    """Proteins with lengths uniform in [len_lo, len_hi] and i.i.d. uniform residues."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(len_lo, len_hi + 1, size=n_proteins)
    total = int(lens.sum())
    res = np.frombuffer(AMINO, dtype=np.uint8)[rng.integers(0, 20, size=total)]
    off = np.zeros(n_proteins + 1, dtype=np.uint64)
    np.cumsum(lens, out=off[1:])
    return Proteome(np.ascontiguousarray(res), off)


def _tryptic_peptides(prot: Proteome, missed: int, min_len: int, max_len: int):
    """(protein, start, length) of tryptic peptides, for picking spectrum sources."""
    res = prot.residues
    n_all = res.shape[0]
    kr = (res == ord("K")) | (res == ord("R"))
    nxt_p = np.zeros(n_all, dtype=bool)
    nxt_p[:-1] = res[1:] == ord("P")
    cut_after = kr & ~nxt_p
    out_p, out_s, out_l = [], [], []
    for i in range(prot.n):
        a, b = int(prot.offsets[i]), int(prot.offsets[i + 1])
        sites = np.nonzero(cut_after[a:b - 1])[0] + 1   # boundaries strictly inside
        bounds = np.concatenate([[0], sites, [b - a]])
        nb = len(bounds)
        for k in range(missed + 1):
            if nb - 1 - k <= 0:
                break
            starts = bounds[:nb - 1 - k]
            ends = bounds[1 + k:]
            ln = ends - starts
            ok = (ln >= min_len) & (ln <= max_len)
            if ok.any():
                out_p.append(np.full(int(ok.sum()), i, dtype=np.int64))
                out_s.append(starts[ok].astype(np.int64))
                out_l.append(ln[ok].astype(np.int64))
    if not out_p:
        z = np.zeros(0, np.int64)
        return z, z, z
    return np.concatenate(out_p), np.concatenate(out_s), np.concatenate(out_l)


def _pick_mod_deltas(rng, seq: bytes, at_nterm: bool, mods: list[Mod], max_mods: int) -> np.ndarray:
    """Per-residue extra mass (float Da) for one random modified form of seq."""
    sites = []  # (position, delta)
    for m in mods:
        if m.nterm:
            if at_nterm:
                sites.append((0, m.delta_da))
        else:
            for j, ch in enumerate(seq):
                if chr(ch) in m.residues:
                    sites.append((j, m.delta_da))
    extra = np.zeros(len(seq), dtype=np.float64)
    if sites and max_mods > 0:
        k = int(rng.integers(0, min(max_mods, len(sites)) + 1))
        if k:
            for s in rng.choice(len(sites), size=k, replace=False):
                extra[sites[s][0]] += sites[s][1]
    return extra


@dataclass
class SpectraRecipe:
    n: int
    charges: tuple = (2,)
    keep_prob: float = 0.6
    mz_sigma: float = 0.005
    n_noise_peaks: tuple = (50, 50)        # inclusive range for real spectra
    noise_frac: float = 0.0                # fraction of pure-noise spectra
    noise_only_peaks: tuple = (50, 100)    # inclusive range for pure-noise spectra
    frag_charge2_for_z3: bool = False      # charge-3 precursors also get 2+ fragments
    peak_count: tuple | None = None        # total peaks per spectrum (uniform), fill with noise
    mass_lognormal: tuple | None = None    # (median Da, sigma): choose source nearest this mass
    mz_lo: float = 100.0
    mz_hi: float = 2000.0


def make_spectra(prot: Proteome, missed: int, min_len: int, max_len: int,
                 mods: list[Mod], max_mods: int, recipe: SpectraRecipe,
                 seed: int = 1) -> Spectra:
    """Spectra drawn from random tryptic peptides of ``prot`` (see module doc)."""
    rng = np.random.default_rng(seed)
    pp, ps, pl = _tryptic_peptides(prot, missed, min_len, max_len)
    if len(pp) == 0:
        raise ValueError("proteome digests to no peptides")
    base_mass = None
    if recipe.mass_lognormal is not None or recipe.noise_frac > 0:
        # float Da base masses, only to pick sources near a drawn mass and to
        # give noise spectra realistic precursor masses
        csum = np.concatenate([[0.0], np.cumsum(_RES_LUT[prot.residues])])
        a = prot.offsets[pp].astype(np.int64) + ps
        base_mass = csum[a + pl] - csum[a] + _WATER_DA
        order = np.argsort(base_mass, kind="stable")
        sorted_mass = base_mass[order]

    n = recipe.n
    is_noise = rng.random(n) < recipe.noise_frac
    charges = np.asarray(recipe.charges, dtype=np.int64)
    z_all = charges[rng.integers(0, len(charges), size=n)]
    mz_parts, in_parts, counts = [], [], np.zeros(n, dtype=np.int64)
    prec = np.zeros(n, dtype=np.float64)
    for s in range(n):
        z = int(z_all[s])
        if is_noise[s]:
            k = int(rng.integers(recipe.noise_only_peaks[0], recipe.noise_only_peaks[1] + 1))
            mz = rng.uniform(recipe.mz_lo, recipe.mz_hi, size=k)
            inten = rng.lognormal(0.0, 1.0, size=k)
            m = float(base_mass[int(rng.integers(0, len(base_mass)))])
        else:
            if recipe.mass_lognormal is not None:
                target = recipe.mass_lognormal[0] * np.exp(recipe.mass_lognormal[1] * rng.standard_normal())
                j = int(np.searchsorted(sorted_mass, target))
                j = min(max(j, 0), len(sorted_mass) - 1)
                if j > 0 and abs(sorted_mass[j - 1] - target) <= abs(sorted_mass[j] - target):
                    j -= 1
                pid = int(order[j])
            else:
                pid = int(rng.integers(0, len(pp)))
            a = int(prot.offsets[pp[pid]]) + int(ps[pid])
            seq = prot.residues[a:a + int(pl[pid])].tobytes()
            extra = _pick_mod_deltas(rng, seq, int(ps[pid]) == 0, mods, max_mods)
            r = _RES_LUT[np.frombuffer(seq, dtype=np.uint8)] + extra
            pre = np.cumsum(r)
            m = float(pre[-1] + _WATER_DA)
            b = pre[:-1] + _PROTON_DA
            y = (pre[-1] - pre[:-1]) + _WATER_DA + _PROTON_DA
            ions = np.concatenate([b, y])
            frag = ions[rng.random(ions.shape[0]) < recipe.keep_prob]
            if recipe.frag_charge2_for_z3 and z >= 3:
                ions2 = (ions + _PROTON_DA) / 2.0
                frag = np.concatenate([frag, ions2[rng.random(ions2.shape[0]) < recipe.keep_prob]])
            frag = frag + rng.normal(0.0, recipe.mz_sigma, size=frag.shape[0])
            if recipe.peak_count is not None:
                total = int(rng.integers(recipe.peak_count[0], recipe.peak_count[1] + 1))
                fi = rng.lognormal(0.0, 1.0, size=frag.shape[0])
                if frag.shape[0] > total:
                    keep = np.argsort(-fi, kind="stable")[:total]
                    frag, fi = frag[keep], fi[keep]
                k = total - frag.shape[0]
                mz = np.concatenate([frag, rng.uniform(recipe.mz_lo, recipe.mz_hi, size=k)])
                inten = np.concatenate([fi, rng.lognormal(0.0, 1.0, size=k)])
            else:
                k = int(rng.integers(recipe.n_noise_peaks[0], recipe.n_noise_peaks[1] + 1))
                mz = np.concatenate([frag, rng.uniform(recipe.mz_lo, recipe.mz_hi, size=k)])
                inten = rng.lognormal(0.0, 1.0, size=mz.shape[0])
        o = np.argsort(mz, kind="stable")
        mz_parts.append(mz[o].astype(np.float32))
        in_parts.append(inten[o].astype(np.float32))
        counts[s] = mz.shape[0]
        prec[s] = (m + z * _PROTON_DA) / z
    off = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=off[1:])
    return Spectra(off, np.concatenate(mz_parts) if mz_parts else np.zeros(0, np.float32),
                   np.concatenate(in_parts) if in_parts else np.zeros(0, np.float32),
                   prec, z_all.astype(np.int8), is_noise)


def poisson_arrivals(n_requests: int, rate_per_s: float, size_lo: int, size_hi: int,
                     seed: int = 2) -> tuple[np.ndarray, np.ndarray]:
    """Arrival times (s, from 0) and batch sizes (uniform in [size_lo, size_hi])."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    sizes = rng.integers(size_lo, size_hi + 1, size=n_requests)
    return t, sizes


# --------------------------------------------------------------------------
# Workload descriptions.  Each names its database and search settings in the
# units the boundary takes (integer micro-Dalton for masses and windows).
# --------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    n_proteins: int
    missed: int
    min_len: int
    max_len: int
    mods: list
    max_mods: int
    recipe: SpectraRecipe
    window_is_ppm: bool
    window: int                 # ppm, or micro-Dalton
    frag_tol_bins: int          # fragment tolerance in 0.01-Da bins
    top_peaks: int
    top_k: int = 5
    min_shared: int = 4
    proteome_seed: int = 0
    spectra_seed: int = 1

    def proteome(self) -> Proteome:
        return make_proteome(self.n_proteins, self.proteome_seed)

    def spectra(self, prot: Proteome | None = None, n: int | None = None, seed: int | None = None,
                charges: tuple | None = None) -> Spectra:
        """The workload's spectra recipe with n spectra; `charges` overrides the
        precursor charges drawn (the serving requests of the large workload use
        2-4)."""
        prot = prot if prot is not None else self.proteome()
        rec = SpectraRecipe(**{**self.recipe.__dict__, **({"n": n} if n is not None else {}),
                               **({"charges": tuple(charges)} if charges is not None else {})})
        return make_spectra(prot, self.missed, self.min_len, self.max_len, self.mods,
                            self.max_mods, rec, self.spectra_seed if seed is None else seed)


def workload(name: str) -> Workload:
    """The named synthetic workloads (tiny closed search through the one-node share)."""
    if name == "tiny":          # 500 proteins, closed search, no mods
        return Workload("tiny", 500, 1, 7, 30, [], 0,
                        SpectraRecipe(n=1000, charges=(2,), n_noise_peaks=(50, 50)),
                        True, 10, 2, 100)
    if name == "medium":        # 20k proteins, open search, Met oxidation
        return Workload("medium", 20000, 2, 7, 40, [OXIDATION], 2,
                        SpectraRecipe(n=100000, charges=(2, 3), n_noise_peaks=(50, 50),
                                      noise_frac=0.2, noise_only_peaks=(50, 100),
                                      frag_charge2_for_z3=True),
                        False, 500_000_000, 1, 100)
    if name == "large":         # 20k proteins, Met-ox + STY phospho, <=3 mods, uneven spectra
        return Workload("large", 20000, 2, 7, 40, [OXIDATION, PHOSPHO], 3,
                        SpectraRecipe(n=1000000, charges=(2, 3), peak_count=(20, 200),
                                      mass_lognormal=(1800.0, 0.25), frag_charge2_for_z3=True),
                        False, 500_000_000, 1, 200)
    if name == "node":          # 200k proteins, four modification types, <=3 mods: one node's share is a partition
        return Workload("node", 200000, 2, 7, 40, [OXIDATION, PHOSPHO, ACETYL_NTERM, DEAMIDATION], 3,
                        SpectraRecipe(n=5000000, charges=(2, 3, 4), peak_count=(20, 200),
                                      mass_lognormal=(1800.0, 0.25), frag_charge2_for_z3=True),
                        False, 500_000_000, 1, 200)
    raise KeyError(name)

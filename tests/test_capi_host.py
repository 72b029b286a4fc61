"""C-ABI library checks that need no GPU: exported symbols, the host-built
index against the oracle's database, and error paths."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth
from paper_2102_02286_amd.capi import ptr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "pepscan.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(ps_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _header_functions()
    assert len(names) >= 15
    L = C.CDLL(capi.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    bound = {s[0] for s in capi._SIGS}
    assert set(names) == bound, set(names) ^ bound


def test_struct_layouts_match_header_sizes():
    assert C.sizeof(capi.ps_device) == 24
    assert C.sizeof(capi.ps_mod) == 24
    assert C.sizeof(capi.ps_db_params) == 48
    assert C.sizeof(capi.ps_part) == 32
    assert capi.SAMPLED_DTYPE.itemsize == 256
    assert C.sizeof(capi.ps_spectra) == 48
    assert C.sizeof(capi.ps_search_params) == 56
    assert capi.HIT_DTYPE.itemsize == 24 and capi.STAT_DTYPE.itemsize == 32


def _both(prot, missed, min_len, max_len, mods, max_mods):
    o = oracle.Database(prot.residues, prot.offsets, missed, min_len, max_len,
                        oracle.mods_from_synth(mods), max_mods)
    h = engine.HostIndex(prot.residues, prot.offsets, missed, min_len, max_len,
                         engine.mods_from_synth(mods), max_mods)
    return o, h


@pytest.mark.parametrize("mods,max_mods", [([], 0), ([synth.OXIDATION], 2),
                                           ([synth.OXIDATION, synth.PHOSPHO, synth.ACETYL_NTERM,
                                             synth.DEAMIDATION], 3)])
def test_host_index_entries_match_oracle(mods, max_mods):
    prot = synth.make_proteome(60, seed=3)
    o, h = _both(prot, 2, 7, 40, mods, max_mods)
    assert len(o) == len(h)
    tab = o.table()
    rng = np.random.default_rng(0)
    for pid in list(range(min(len(o), 200))) + list(rng.integers(0, len(o), 500)):
        pid = int(pid)
        assert h.entry(pid) == tuple(int(x) for x in tab[pid]), pid


def test_host_index_postings_match_oracle_ions():
    """CSR postings equal bins of the oracle's b/y ions, listed in id order."""
    prot = synth.make_proteome(25, seed=4)
    mods = [synth.OXIDATION, synth.PHOSPHO]
    o, h = _both(prot, 1, 7, 30, mods, 2)
    off, post = h.host_arrays()
    want = {}
    for pid in range(len(o)):
        b, y = oracle.ions(o.residue_masses(pid))
        for m in b:
            want.setdefault(int((m + 5000) // 10000), []).append(pid << 1)
        for m in y:
            want.setdefault(int((m + 5000) // 10000), []).append(pid << 1 | 1)
    assert int(off[-1]) == post.shape[0] == sum(len(v) for v in want.values())
    for bn in range(off.shape[0] - 1):
        got = post[off[bn]:off[bn + 1]].tolist()
        assert got == sorted(want.get(bn, [])), bn


def test_peptide_strings():
    prot = synth.Proteome(np.frombuffer(b"MSTKPEPTIDER", np.uint8).copy(), np.array([0, 12], np.uint64))
    h = engine.HostIndex(prot.residues, prot.offsets, 1, 4, 20,
                         engine.mods_from_synth([synth.PHOSPHO, synth.ACETYL_NTERM]), 2)
    strings = {h.peptide(i) for i in range(len(h))}
    assert "MSTKPEPTIDER" in strings
    assert "n[+42.010565]MS[+79.966331]TKPEPTIDER" in strings
    assert "MST[+79.966331]KPEPTIDER" in strings


def test_index_create_rejects_bad_input():
    bad = synth.Proteome(np.frombuffer(b"PEPXIDEK", np.uint8).copy(), np.array([0, 8], np.uint64))
    with pytest.raises(capi.PsError) as e:
        engine.HostIndex(bad.residues, bad.offsets, 1, 4, 20, [], 0)
    assert e.value.code == capi.PS_EINVAL
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEK", np.uint8).copy(), np.array([0, 8], np.uint64))
    with pytest.raises(capi.PsError):
        engine.HostIndex(ok.residues, ok.offsets, 1, 10, 5, [], 0)             # min_len > max_len
    with pytest.raises(capi.PsError):
        engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20,
                         [engine.Mod("ST", 1), engine.Mod("TY", 2)], 1)        # T in two mods
    with pytest.raises(capi.PsError) as e:
        engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [engine.Mod("G", -56_500_000)], 1)   # G -> 0.5 Da
    assert "lighter" in str(e.value)


def test_no_device_is_reported_not_crashed():
    """In a container without a GPU, upload and search fail with PS_EDEVICE."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEKAAAAR", np.uint8).copy(), np.array([0, 13], np.uint64))
    h = engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [], 0)
    dev = capi.ps_device(None, 0, None)
    rc = capi.ps_index_upload(h.handle, C.byref(dev))
    assert rc == capi.PS_EDEVICE
    assert "device" in capi.last_error()


def test_search_params_validation_without_device():
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEKAAAAR", np.uint8).copy(), np.array([0, 13], np.uint64))
    h = engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [], 0)
    need = C.c_uint64()
    for bad in [engine.search_params(False, 1, 1, 100, top_k=0),
                engine.search_params(False, 1, 1, 100, top_k=17),
                engine.search_params(False, 1, 9, 100),
                engine.search_params(False, -1, 1, 100),
                engine.search_params(False, 1, 1, 100, min_shared=0),
                engine.search_params(False, 1, 1, 256, max_charge=8),          # too many segments
                engine.search_params(True, 2_000_000, 1, 100),
                engine.search_params(False, 1, 1, 100, fit=2),
                engine.search_params(False, 1, 1, 100, noise_permille=1001),
                engine.search_params(False, 1, 1, 100, intensity=2)]:
        assert capi.ps_workspace_bytes(h.handle, 10, 100, C.byref(bad), C.byref(need)) == capi.PS_EINVAL
    good = engine.search_params(False, 1, 1, 100, max_charge=3)
    assert capi.ps_workspace_bytes(h.handle, 10, 100, C.byref(good), C.byref(need)) == capi.PS_OK
    assert need.value > 10 * 512 * 4


def test_schedule_validation_and_tile_directory():
    prot = synth.make_proteome(30, seed=5)
    h = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, [], 0)
    grain, nbytes = h.directory()
    assert grain == 12
    n_pep, n_post, n_bins = h.shape()
    assert nbytes == n_bins * (((n_pep >> 12) + 2 + 3) // 4 * 4) * 4
    assert h.schedule().tile >= 1 << grain
    for bad in [dict(tile=2048), dict(tile=6144), dict(tile=65536), dict(tiles_per_item=0), dict(groups_per_cu=9),
                dict(group_threads=384), dict(group_threads=512, tile=4096)]:
        with pytest.raises(capi.PsError) as e:
            h.set_schedule(**bad)
        assert e.value.code == capi.PS_EINVAL
    sc = h.schedule()
    sc.reserved[1] = 7
    assert capi.ps_index_set_schedule(h.handle, C.byref(sc)) == capi.PS_EINVAL
    h.set_schedule(tile=8192, tiles_per_item=7, groups_per_cu=3)
    got = h.schedule()
    assert (got.tile, got.tiles_per_item, got.groups_per_cu) == (8192, 7, 3)
    h.set_schedule(group_threads=512)
    assert h.schedule().group_threads == 512


def test_dense_maps_exist_only_on_the_device():
    """Dense maps are built when the index goes to the device; a host index
    has none, and the switch that stops searches reading them is kept."""
    prot = synth.make_proteome(40, seed=2)
    h = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, [], 0)
    bins, on = h.dense()
    assert bins.size == 0 and on
    h.set_dense(False)
    assert h.dense()[1] is False
    h.set_dense(True)
    assert h.dense()[1] is True
    assert capi.ps_index_dense(None, None, None, None) == capi.PS_EINVAL
    assert capi.ps_index_set_dense(None, 0) == capi.PS_EINVAL


def test_tile_directory_matches_postings():
    """dir[bin][k] is the position, inside the bin's own list, of the first
    posting whose id is >= k * 4096 (rows padded to a multiple of four
    entries, the padding repeating the list's length)."""
    prot = synth.make_proteome(400, seed=6)
    h = engine.HostIndex(prot.residues, prot.offsets, 2, 7, 30, engine.mods_from_synth([synth.OXIDATION]), 2)
    n_pep, _, n_bins = h.shape()
    assert n_pep > 3 * 4096
    off, post = h.host_arrays()
    d = h.directory_array()
    nblk = (n_pep >> 12) + 1
    stride = (nblk + 1 + 3) // 4 * 4
    assert d.shape == (n_bins, stride)
    rng = np.random.default_rng(1)
    for bn in list(rng.integers(0, n_bins, 300)) + [int(np.argmax(np.diff(off.astype(np.int64))))]:
        ids = post[off[bn]:off[bn + 1]] >> 1
        want = np.searchsorted(ids, np.arange(stride) * 4096, side="left")
        assert np.array_equal(d[bn].astype(np.uint64), want.astype(np.uint64)), bn


def test_server_and_plan_need_an_uploaded_index():
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEKAAAAR", np.uint8).copy(), np.array([0, 13], np.uint64))
    h = engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [], 0)
    prm = engine.search_params(False, 1000, 1, 50, max_charge=3, schedule=capi.PS_SCHED_PERSISTENT)
    dev = capi.ps_device(None, 0, None)
    out = C.c_void_p()
    rc = capi.ps_plan_create(h.handle, C.byref(dev), 10, 100, C.byref(prm), C.byref(out))
    assert rc in (capi.PS_EDEVICE, capi.PS_EINVAL) and not out.value
    rc = capi.ps_server_create(h.handle, C.byref(dev), C.byref(prm), 10, 100, 2, 0, C.byref(out))
    assert rc in (capi.PS_EDEVICE, capi.PS_EINVAL, capi.PS_ENOMEM) and not out.value
    # argument checks come before the device check
    assert capi.ps_server_create(h.handle, C.byref(dev), C.byref(prm), 10, 100, 0, 0, C.byref(out)) == capi.PS_EINVAL
    assert capi.ps_server_create(h.handle, C.byref(dev), C.byref(prm), 0, 100, 2, 0, C.byref(out)) == capi.PS_EINVAL


@pytest.mark.parametrize("T", [1, 2])
def test_merged_lists_are_neighbour_unions(T):
    """With merge width T the list of bin b is the id-ordered union of the
    classic lists of bins b-T..b+T; searches must use that tolerance."""
    prot = synth.make_proteome(40, seed=7)
    mods = engine.mods_from_synth([synth.OXIDATION])
    classic = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, mods, 2)
    merged = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, mods, 2, merge_tol=T)
    oc, pc = classic.host_arrays()
    om, pm = merged.host_arrays()
    nb = oc.shape[0] - 1
    assert om.shape == oc.shape and pm.shape[0] <= (2 * T + 1) * pc.shape[0]
    for bn in range(nb):
        parts = [pc[oc[b]:oc[b + 1]] for b in range(max(0, bn - T), min(nb, bn + T + 1))]
        want = np.sort(np.concatenate(parts)) if parts else np.zeros(0, np.uint32)
        assert np.array_equal(pm[om[bn]:om[bn + 1]], want), bn
    # the tile directory indexes the merged lists
    d = merged.directory_array()
    for bn in range(0, nb, 97):
        ids = pm[om[bn]:om[bn + 1]] >> 1
        assert np.array_equal(d[bn], np.searchsorted(ids, np.arange(d.shape[1]) * 4096))
    need = C.c_uint64()
    wrong = engine.search_params(False, 1000, T + 1, 100, max_charge=3)
    assert capi.ps_workspace_bytes(merged.handle, 10, 100, C.byref(wrong), C.byref(need)) == capi.PS_EINVAL
    assert "frag_tol_bins" in capi.last_error()
    right = engine.search_params(False, 1000, T, 100, max_charge=3)
    assert capi.ps_workspace_bytes(merged.handle, 10, 100, C.byref(right), C.byref(need)) == capi.PS_OK
    with pytest.raises(capi.PsError):
        engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, mods, 2, merge_tol=5)


@pytest.mark.parametrize("G,T", [(2, 0), (3, 0), (3, 2)])
def test_partition_index_is_a_round_robin_slice(G, T):
    """Partition g of G holds whole-database entries g, g + G, ... in order; its
    postings are the whole index's postings of those entries with ids divided by
    G, bin by bin, over the same bin range (merged lists included)."""
    prot = synth.make_proteome(40, seed=5)
    mods = engine.mods_from_synth([synth.OXIDATION])
    whole = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, mods, 1, merge_tol=T)
    ow, pw = whole.host_arrays()
    n_whole = len(whole)
    total_post = 0
    for g in range(G):
        part = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, mods, 1, merge_tol=T, n_shards=G, shard=g)
        n_pep, n_post, n_bins = part.shape()
        assert n_pep == len(range(g, n_whole, G)) and n_bins == whole.shape()[2]
        for i in list(range(min(n_pep, 50))) + [n_pep - 1]:
            assert part.entry(i) == whole.entry(i * G + g)
        op, pp = part.host_arrays()
        total_post += n_post
        for bn in range(0, n_bins, 7):
            w = pw[ow[bn]:ow[bn + 1]]
            ids = w >> 1
            keep = w[ids % G == g]
            want = ((keep >> 1) // G) << 1 | (keep & 1)
            assert np.array_equal(pp[op[bn]:op[bn + 1]], want.astype(np.uint32)), (g, bn)
    assert total_post == pw.shape[0]


def test_partition_and_assemble_argument_checks_without_device():
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEKAAAAR", np.uint8).copy(), np.array([0, 13], np.uint64))
    for G, g in [(2, 2), (65, 0)]:
        with pytest.raises(capi.PsError) as e:
            engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [], 0, n_shards=G, shard=g)
        assert e.value.code == capi.PS_EINVAL
    # a partition with no entries at all is valid
    empty = engine.HostIndex(ok.residues, ok.offsets, 1, 4, 20, [], 0, n_shards=64, shard=63)
    assert len(empty) == 0
    parts = (capi.ps_part * 2)()
    assert capi.ps_assemble(None, 0, parts, 1, 5, 0, 1, 1, 1) == capi.PS_EINVAL
    assert capi.ps_assemble(None, 65, parts, 1, 5, 0, 1, 1, 1) == capi.PS_EINVAL
    assert capi.ps_assemble(None, 2, parts, 1, 0, 0, 1, 1, 1) == capi.PS_EINVAL
    assert capi.ps_assemble(None, 2, parts, 1, 17, 0, 1, 1, 1) == capi.PS_EINVAL
    assert capi.ps_assemble(None, 2, parts, 1, 5, 2, 1, 1, 1) == capi.PS_EINVAL     # unknown fit
    assert capi.ps_assemble(None, 2, parts, 1, 5, 0, 1, 1, 1) == capi.PS_EINVAL     # NULL partition pointers
    assert "partition 0" in capi.last_error()
    # exactly one of the full and the sampled histograms
    parts[0] = capi.ps_part(8, 8, 8, 8)
    parts[1] = capi.ps_part(8, 8, 8, None)
    assert capi.ps_assemble(None, 2, parts, 1, 5, 0, 1, 1, 1) == capi.PS_EINVAL
    assert "exactly one of hist and sampled" in capi.last_error()
    parts[0] = capi.ps_part(8, 8, None, None)
    assert capi.ps_assemble(None, 2, parts, 1, 5, 0, 1, 1, 1) == capi.PS_EINVAL
    assert "exactly one of hist and sampled" in capi.last_error()
    assert capi.ps_assemble(None, 2, parts, 0, 5, 0, None, None, None) == capi.PS_OK  # nothing to do
    # sampling: NULL pointers are rejected before any device work; nothing to do is fine
    assert capi.ps_sample(None, 1, None, 8, 8) == capi.PS_EINVAL
    assert capi.ps_sample(None, 1, 8, None, 8) == capi.PS_EINVAL
    assert capi.ps_sample(None, 1, 8, 8, None) == capi.PS_EINVAL
    assert capi.ps_sample(None, 0, None, None, None) == capi.PS_OK


def test_bulk_entries_match_single_entries():
    prot = synth.make_proteome(20, seed=8)
    h = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, engine.mods_from_synth([synth.OXIDATION]), 2)
    tab = h.entries()
    for pid in range(0, len(h), 37):
        assert h.entry(pid) == tuple(int(x) for x in tab[pid])
    assert capi.ps_index_entries(h.handle, len(h), 1, None, None, None, None, None) == capi.PS_EINVAL
    assert capi.ps_index_entries(h.handle, len(h), 0, None, None, None, None, None) == capi.PS_OK


def test_device_build_without_device():
    """The device build checks its arguments like ps_index_create, then needs a GPU."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    ok = synth.Proteome(np.frombuffer(b"PEPTIDEKAAAAR", np.uint8).copy(), np.array([0, 13], np.uint64))
    p, keep = engine._db_params(1, 4, 20, [], 0)
    a, b = C.c_uint64(), C.c_uint64()
    assert capi.ps_index_build_device_bytes(C.byref(p), ptr(ok.residues), ptr(ok.offsets), 1, 0, C.byref(a),
                                            C.byref(b)) == capi.PS_EDEVICE
    bad, keep2 = engine._db_params(1, 10, 5, [], 0)            # min_len > max_len
    assert capi.ps_index_build_device_bytes(C.byref(bad), ptr(ok.residues), ptr(ok.offsets), 1, 0, C.byref(a),
                                            C.byref(b)) == capi.PS_EINVAL
    dev = capi.ps_device(None, 0, None)
    out = C.c_void_p()
    assert capi.ps_index_build_device(C.byref(p), ptr(ok.residues), ptr(ok.offsets), 1, 0, C.byref(dev),
                                      C.byref(dev), C.byref(out)) == capi.PS_EDEVICE
    assert not out.value


@pytest.mark.parametrize("types,label", [(63, "abcxyz"), (4 | 32, "cz"), (1 | 8, "ax")])
def test_host_index_postings_other_ion_series(types, label):
    """Postings of the a, c, x, z series: the oracle's b/y ions shifted by the
    element-derived offsets; N-terminal series carry bit 0, C-terminal bit 1."""
    from tests import bruteforce as bf
    prot = synth.make_proteome(20, seed=9)
    mods = [synth.OXIDATION, synth.ACETYL_NTERM]
    o = oracle.Database(prot.residues, prot.offsets, 1, 7, 30, oracle.mods_from_synth(mods), 1)
    h = engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, engine.mods_from_synth(mods), 1, ion_types=types)
    off, post = h.host_arrays()
    want = {}
    for pid in range(len(o)):
        b, y = oracle.ions(o.residue_masses(pid))
        for t in label:
            base, flag = (b, 0) if t in "abc" else (y, 1)
            for m in base:
                want.setdefault(int((m + bf.ION_SHIFT[t] + 5000) // 10000), []).append(pid << 1 | flag)
    assert int(off[-1]) == post.shape[0] == sum(len(v) for v in want.values())
    for bn in range(off.shape[0] - 1):
        assert post[off[bn]:off[bn + 1]].tolist() == sorted(want.get(bn, [])), bn
    with pytest.raises(capi.PsError):
        engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, [], 0, ion_types=64)
    with pytest.raises(capi.PsError):     # a ions need residues heavier than CO
        engine.HostIndex(prot.residues, prot.offsets, 1, 7, 30, [engine.Mod("G", -30_000_000)], 1, ion_types=1)

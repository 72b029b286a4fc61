"""One node's share of the largest database (needs an MI355X).

The database: 200k proteins, up to two missed cleavages, length 7-40,
oxidation, STY phosphorylation, protein N-terminal acetylation and N/Q
deamidation with at most three modified sites per peptide -- 1.12G peptides,
63.7G b/y postings.  The paper spreads its largest database (3.88G entries)
over 64 nodes, about 61M entries each; here one GPU holds partition 0 of 16
round-robin partitions of the sorted database (70M peptides, 11.9G postings in
lists merging three neighbouring bins, built on the GPU).  The oracle digests
and sorts the whole database itself, takes the same partition, and scores
every window candidate of sampled spectra by generating its ions.
"""
import numpy as np
import pytest

import oracle
from paper_2102_02286_amd import capi, engine, synth
from tests.test_gpu_parity import assert_parity

pytestmark = pytest.mark.gpu

G, SHARD = 16, 0


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def node():
    w = synth.workload("node")
    prot = w.proteome()
    _say("node share: building partition 0 of 16 on the GPU")
    ix = engine.HostIndex.build_on_device(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                                          engine.mods_from_synth(w.mods), w.max_mods, merge_tol=w.frag_tol_bins,
                                          n_shards=G, shard=SHARD)
    n_pep, n_post, n_bins = ix.shape()
    _say(f"node share: {n_pep} peptides, {n_post} postings; oracle database of the whole proteome")
    whole = oracle.Database(prot.residues, prot.offsets, w.missed, w.min_len, w.max_len,
                            oracle.mods_from_synth(w.mods), w.max_mods)
    _say(f"node share: oracle holds {len(whole)} peptides; taking partition {SHARD} of {G}")
    db = whole.shard(G, SHARD)
    total = len(whole)
    del whole
    assert len(db) == n_pep
    return w, prot, ix, db, total


def test_node_share_shape_and_entries(node):
    w, prot, ix, db, total = node
    n_pep, n_post, n_bins = ix.shape()
    assert total > 1_000_000_000 and n_pep == (total - SHARD + G - 1) // G
    assert n_post > 1 << 33
    rng = np.random.default_rng(5)
    ent = ix.entries()
    for i in np.concatenate([rng.integers(0, n_pep, 300), [0, n_pep - 1]]):
        assert tuple(ent[int(i)]) == db.get(int(i))


@pytest.mark.parametrize("schedule,sched", [(capi.PS_SCHED_PLAIN, dict(tile=8192, group_threads=512)),
                                            (capi.PS_SCHED_PERSISTENT, dict(tile=8192, group_threads=512,
                                                                            tiles_per_item=128, groups_per_cu=3))])
def test_node_share_sampled_parity(node, schedule, sched):
    """2000 spectra of the serving recipe (charges 2-4) searched on the
    partition; 16 of them against the oracle's partition."""
    w, prot, ix, db, total = node
    sp = w.spectra(prot, n=2000, seed=51)
    ix.set_schedule(**sched)
    prm = engine.search_params(w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared,
                               max_charge=4, schedule=schedule)
    _say(f"node share: searching {sp.n} spectra, schedule {schedule}")
    res = engine.search(ix, sp, prm)
    assert res.overflow_spectra == 0
    idx = np.sort(np.random.default_rng(6).choice(sp.n, 16, replace=False))
    sub = sp.subset(idx)
    _say("node share: oracle on 16 sampled spectra")
    oh, ost, og = db.search(sub, w.window_is_ppm, w.window, w.frag_tol_bins, w.top_peaks, w.top_k, w.min_shared)
    from types import SimpleNamespace
    assert_parity(SimpleNamespace(hits=res.hits[idx], stats=res.stats[idx], hist=res.hist[idx]), oh, ost, og)
    assert (ost["status"] == 0).sum() >= 10

"""Batched persistent traversal (one launch, device work queue, HIP-graph replay)
versus the CPU oracle, network by network: bit-exact pathway sets, flux vectors
and status flags."""
import numpy as np
import pytest

import oracle
from invariants import check_result
from paper_1804_02867_amd import netgen

pytestmark = pytest.mark.gpu

efm = pytest.importorskip("paper_1804_02867_amd.efm")


def _oracle(net, x, D, cap):
    S, rev, ext = net.arrays()
    return oracle.enumerate_pathways(S, rev, ext, x, depth_cap=D, frontier_cap=cap)


def _check_all(batch, nets, targets, D, cap):
    for i, (net, x) in enumerate(zip(nets, targets)):
        got = batch.result(i)
        want = _oracle(net, x, D, cap)
        assert got.status == want.status, f"network {i} ({net.name}) target {x}"
        assert np.array_equal(got.keys, want.keys), f"network {i} ({net.name}) target {x}"
        assert np.array_equal(got.flux, want.flux), f"network {i} ({net.name}) target {x}"
        assert got.levels[0]["parents"] == int(want.levels[:, 0].sum()) + 1
        check_result(*net.arrays(), x, got.keys, got.flux, D)


def test_batch_members_match_oracle_on_every_replay():
    nets = [netgen.batch_member(i) for i in range(48)]
    targets = [n.targets[0] for n in nets]
    D, cap = 10, 3000
    print(f"case batch 48 members D={D} cap={cap}", flush=True)
    handles = [efm.Network(*n.arrays()) for n in nets]
    b = efm.Batch(handles, targets, depth_cap=D, frontier_cap=cap)
    for replay in range(3):
        b.run()
        _check_all(b, nets, targets, D, cap)
        lat = b.latency_ns()
        assert (lat > 0).all()
    b.close()


def test_batch_full_enumeration_of_tiny_networks():
    nets, targets = [], []
    for seed in range(8):
        net = netgen.tiny(seed)
        for x in net.targets:
            nets.append(net)
            targets.append(x)
    nets.append(netgen.diamonds(6))
    targets.append(nets[-1].targets[-1])
    print(f"case batch tiny x{len(nets)} full", flush=True)
    handles = [efm.Network(*n.arrays()) for n in nets]
    b = efm.Batch(handles, targets)
    b.run()
    _check_all(b, nets, targets, 0, 0)
    assert b.result(len(nets) - 1).count == 64
    b.close()


def test_batch_autotune_and_options_change_nothing():
    nets = [netgen.batch_member(i) for i in range(48, 72)]
    targets = [n.targets[-1] for n in nets]
    D, cap = 9, 500
    handles = [efm.Network(*n.arrays()) for n in nets]
    for flags in (efm.OPT_AUTOTUNE, efm.OPT_NO_GF2, efm.OPT_EXACT_RANK | efm.OPT_NO_PRUNE):
        print(f"case batch flags={flags}", flush=True)
        b = efm.Batch(handles, targets, depth_cap=D, frontier_cap=cap, flags=flags)
        wpn, npc = b.config()
        assert wpn in (1, 2, 4, 8) and npc >= 1
        b.run()
        _check_all(b, nets, targets, D, cap)
        b.close()


def test_batch_rejects_bad_input():
    net = netgen.tiny(0)
    h = efm.Network(*net.arrays())
    with pytest.raises(efm.EfmError) as e:
        efm.Batch([h], [0])                            # internal metabolite
    assert e.value.code == efm.EINVAL
    big = efm.Network(*netgen.genome(0).arrays())
    with pytest.raises(efm.EfmError) as e:
        efm.Batch([big], [netgen.genome(0).targets[0]])   # too large for the batched engine
    assert e.value.code == efm.EINVAL

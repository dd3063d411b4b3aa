"""The partition cache's slot policy (host only, no GPU): its decisions and
the release batch of every upload against a model of the policy, and the
ordering property the release point must satisfy: a slot is overwritten only
after every batch that used it has been enqueued in full, never before."""
import numpy as np
import pytest

from policy_model import RING, Capacity, PolicyModel


@pytest.fixture(scope="module")
def hg():
    import paper_2507_15683_amd as hg
    return hg


def test_release_waits_for_the_batch_after_the_last_use(hg):
    """Two slots, four partitions.  Batch 0 fills both slots (nothing to wait
    for); batch 1 replaces both, so each copy waits for the start of batch 1,
    which follows batch 0's renders -- the renders that read the old data."""
    pol = hg.SlotPolicy(4, 2)
    st = pol.step([1, 1, 0, 0])
    assert st["upload_list"] == [(0, 0, -1, 0), (1, 1, -1, 0)]
    st = pol.step([0, 0, 1, 1])
    assert (st["hits"], st["uploads"], st["evictions"]) == (0, 2, 2)
    assert st["upload_list"] == [(2, 0, 1, 0), (3, 1, 1, 0)]
    # partition 0 comes back into the least recently used slot (slot 0, tie
    # to the lower slot), which batch 1 used: wait for batch 2's start
    st = pol.step([1, 0, 0, 1])
    assert st["upload_list"] == [(0, 0, 2, 0)] and st["hits"] == 1
    pol.close()


def test_release_of_a_long_idle_slot_is_clamped_to_the_ring(hg):
    """A slot last used 20 batches ago waits for the oldest start point the
    ring of 16 still holds (a later, still safe, release)."""
    pol = hg.SlotPolicy(3, 2)
    pol.step([1, 1, 0])          # batch 0: partitions 0, 1
    for _ in range(20):
        pol.step([0, 1, 0])      # batches 1..20: partition 1 only
    st = pol.step([0, 1, 1])     # batch 21: partition 2 evicts 0 (slot 0, idle since batch 0)
    assert st["upload_list"] == [(2, 0, 21 - (RING - 1), 0)]
    pol.close()


def test_policy_follows_the_model_and_never_releases_early(hg):
    """Random batches (rendered and upcoming needs, capacity errors, an
    eviction of everything): counts and upload lists equal the model's, and
    every release lies after the slot's previous use and no later than the
    batch itself."""
    rng = np.random.default_rng(5)
    for n_parts, S in ((16, 4), (16, 5), (9, 9), (40, 7)):
        pol, model = hg.SlotPolicy(n_parts, S), PolicyModel(n_parts, S)
        last_use = [-1] * S
        batch = 0
        for it in range(300):
            need = np.zeros(n_parts, np.uint8)
            need[rng.choice(n_parts, min(n_parts, rng.integers(0, S + 2)), replace=False)] = 1
            up = rng.choice(n_parts, rng.integers(0, 4), replace=False)
            need[up[need[up] == 0]] = 2
            if it == 150:
                pol.evict_all()
                model.evict_all()
            try:
                want = model.step(need)
            except Capacity:
                with pytest.raises(hg.HgsrError, match="CAPACITY"):
                    pol.step(need)
                continue
            got = pol.step(need)
            for f in ("needed", "hits", "uploads", "evictions", "prefetched", "upload_list"):
                assert got[f] == want[f], (n_parts, S, it, f)
            for part, slot, rel, ahead in got["upload_list"]:
                if last_use[slot] < 0:
                    assert rel == -1
                else:
                    assert last_use[slot] < rel <= batch
            for k in np.nonzero(need)[0]:
                s = model.where.get(int(k))
                if s is not None:
                    last_use[s] = batch
            batch += 1
        pol.close()


def test_policy_arguments_rejected(hg):
    with pytest.raises(hg.HgsrError, match="INVALID_ARG"):
        hg.SlotPolicy(4, 5)
    with pytest.raises(hg.HgsrError, match="INVALID_ARG"):
        hg.SlotPolicy(100, 65)
    pol = hg.SlotPolicy(4, 2)
    with pytest.raises(hg.HgsrError, match="INVALID_ARG"):
        pol.step([3, 0, 0, 0])
    pol.close()

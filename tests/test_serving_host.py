"""Host-side logic of the serving loop: class grid, request trace recipe and
arena slot bookkeeping (no GPU needed)."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def sv():
    import paper_1504_07038_amd as mj
    import os

    if not os.path.exists(mj.LIB_PATH):
        from paper_1504_07038_amd import build

        build.build()
    from paper_1504_07038_amd import serving

    return serving


def test_class_grid_covers_4k_to_1m(sv):
    for k in (4, 8):
        g = sv.class_grid(k, 4)
        assert g[0] * 8 * k == 4096 and g[-1] * 8 * k == 1 << 20
        assert len(g) == 33 and all(b > a for a, b in zip(g, g[1:]))
        # consecutive classes differ by 2^(1/4) up to rounding, so an object
        # is padded by under a fifth of its size
        assert all(b <= a * 2 ** 0.25 + 1 for a, b in zip(g, g[1:]))


def test_trace_recipe(sv):
    geos = sv.geometries(per_octave=2)
    tr = sv.make_trace(100000, 0.5, geos, seed=5)
    N = len(tr.arrival)
    assert abs(N - 50000) < 5 * np.sqrt(50000)
    assert (np.diff(tr.arrival) >= 0).all() and tr.arrival[-1] < 0.5
    gaps = np.diff(tr.arrival)
    assert abs(gaps.mean() * 1e5 - 1) < 0.03 and abs(gaps.std() / gaps.mean() - 1) < 0.05
    assert abs(tr.read.mean() - 0.7) < 0.01
    ks = np.array([g.k for g in geos])[tr.cls]
    ms = np.array([g.m for g in geos])[tr.cls]
    Ps = np.array([g.P for g in geos])[tr.cls]
    assert set(np.unique(ks)) == {4, 8}
    assert (tr.size % (8 * ks) == 0).all()
    assert tr.size.min() >= 4096 and tr.size.max() <= 1 << 20
    assert (Ps * ks * 8 >= tr.size).all()
    # the class is the smallest one that fits
    for c, g in enumerate(geos):
        sel = tr.cls == c
        smaller = [h.P for h in geos if (h.k, h.m) == (g.k, g.m) and h.P < g.P]
        if smaller and sel.any():
            assert (tr.size[sel] > max(smaller) * g.k * 8).all()
    # log2 of the size is uniform over [12, 20]
    lg = np.log2(tr.size)
    assert abs(np.median(lg) - 16) < 0.1
    pop = np.array([bin(int(x)).count("1") for x in tr.mask])
    assert (pop <= ms).all()
    for m in (2, 4):
        counts = np.bincount(pop[ms == m], minlength=m + 1)
        assert counts.min() > 0.8 * counts.mean()


def test_slot_store_free_then_oldest_idle(sv):
    st = sv.SlotStore(6)
    rng = np.random.default_rng(0)
    a = st.take_write_slots(4)
    assert sorted(a) == [0, 1, 2, 3] and st.nfree == 2
    st.push_resident(a, np.arange(4))
    held = st.pick_resident(50, rng)
    assert set(held) <= set(a)
    st.release(held)
    assert (st.refs == 0).all()
    b = st.take_write_slots(3)            # two free, then the oldest resident
    assert sorted(b[:2]) == [4, 5] and b[2] == a[0]
    assert st.count == 3 and st.source[a[0]] == -1
    st.push_resident(b, np.arange(10, 13))
    # an in-flight read of the oldest object: it is skipped and moves to
    # the young end; the next oldest idle objects are evicted
    res0 = list(st.resident())
    st.refs[res0[0]] = 1
    c = st.take_write_slots(2)
    assert list(c) == res0[1:3]
    assert list(st.resident()) == res0[3:] + [res0[0]]
    assert st.count == len(res0) - 2
    st.refs[res0[0]] = 0
    res = st.resident()
    assert len(set(res)) == len(res) and not set(res) & set(c)
    # every resident object held: nothing to evict
    st.refs[st.resident()] = 1
    assert len(st.take_write_slots(1)) == 0 and list(st.resident()) == list(res)
    st.refs[:] = 0


def test_slot_store_random_operations_keep_slots_unique(sv):
    """Random writes, reads and releases: every slot is free, resident or in a
    write that has not completed, never two of these; held objects are never
    evicted."""
    st = sv.SlotStore(40)
    rng = np.random.default_rng(5)
    pending_writes, held = [], []
    for _ in range(3000):
        op = rng.integers(0, 4)
        if op == 0:
            got = st.take_write_slots(int(rng.integers(1, 8)))
            assert not set(got.tolist()) & set(np.concatenate(held).tolist() if held else [])
            pending_writes.append(got)
        elif op == 1 and pending_writes:
            w = pending_writes.pop(0)
            st.push_resident(w, np.arange(len(w)))
        elif op == 2 and st.count:
            held.append(st.pick_resident(int(rng.integers(1, 6)), rng))
        elif op == 3 and held:
            st.release(held.pop(0))
        res = st.resident().tolist()
        free = st.free[:st.nfree].tolist()
        inw = np.concatenate(pending_writes).tolist() if pending_writes else []
        assert len(set(res)) == len(res)
        assert not set(res) & set(free) and not set(res) & set(inw) and not set(free) & set(inw)
        assert len(res) + len(free) + len(inw) == st.slots
        assert (st.refs >= 0).all()

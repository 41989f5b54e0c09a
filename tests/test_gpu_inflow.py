"""GPU tests of the time-interpolated inflow (les_set_inflow_pair; section
4, coupled time loop) against the FP64 oracle, which replays the GPU's SOR
iteration counts.  Bar as for the other one-step parity tests: relative L2
per field <= 1e-5 after every step; the interpolated inflow face itself
within 1e-6 (float32 profile and weight against float64)."""
import threading

import numpy as np
import pytest

import oracle
import paper_1504_02264_amd as les
from les_inputs import building_heights, building_mask, log_law_profile
from paper_1504_02264_amd.coupling import CoupledInflow, ProfileFeed

pytestmark = pytest.mark.gpu

NX, NY, NZ, DT = 24, 20, 12, 0.05


def rel(a, b):
    b = np.asarray(b, np.float64)
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def case(seed=3):
    h = building_heights(NX, NY, NZ, 0.15, 2, 4, 2, 6, seed=seed, margin_x=4, margin_y=2)
    mask = building_mask(h, NZ)
    u0 = log_law_profile(NZ, 2.0)
    u1 = (1.3 * u0 + 0.2 * np.linspace(0, 1, NZ)).astype(np.float32)
    return mask, u0, u1


def make(mask):
    return (les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask),
            oracle.Oracle(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask))


def test_interpolated_inflow_matches_oracle():
    """Steps before, inside and after [t0, t1] (t0 = 1 dt, t1 = 5 dt)."""
    print(f"[inflow pair] {NX}x{NY}x{NZ}", flush=True)
    mask, u0, u1 = case()
    g, o = make(mask)
    try:
        for x in (g, o):
            x.set_inflow(u0, 0.01, 3)
            x.set_inflow_pair(1 * DT, u0, 5 * DT, u1)
        for s in range(7):
            _, _, it = g.step(1)
            o.step(1, forced=it)
            a, b = g.get_fields(), o.get_fields()
            face = np.max(np.abs(a[0][..., 0] - b[0][..., 0])) / np.max(np.abs(b[0][..., 0]))
            errs = [rel(x, y) for x, y in zip(a, b)]
            print(f"  step {s}: face {face:.2e} fields {max(errs):.2e}", flush=True)
            assert face <= 1e-6
            assert max(errs) <= 1e-5
        # the run did follow the second sample: the face mean moved towards U1
        assert np.mean(a[0][..., 0]) > 1.2 * np.mean(np.where(mask[:, :, 0] == 0, u0[:, None], 0))
    finally:
        g.close()


def test_pair_of_equal_samples_is_bitwise_the_plain_run():
    mask, u0, _ = case()
    a = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    b = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    try:
        a.set_inflow(u0, 0.01, 3)
        b.set_inflow(u0, 0.01, 3)
        b.set_inflow_pair(0.0, u0, 0.1, u0)
        _, _, ia = a.step(3)
        _, _, ib = b.step(3)
        assert list(ia) == list(ib)
        for x, y in zip(a.get_fields(), b.get_fields()):
            assert np.array_equal(x, y)
    finally:
        a.close()
        b.close()


def test_checkpoint_keeps_the_pair():
    mask, u0, u1 = case()
    ref = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    b = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    c = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    try:
        for x in (ref, b):
            x.set_inflow(u0, 0.01, 3)
            x.set_inflow_pair(0.0, u0, 6 * DT, u1)
        ref.step(6)
        b.step(3)
        c.set_state(b.get_state())
        c.step(3)
        for x, y in zip(ref.get_fields(), c.get_fields()):
            assert np.array_equal(x, y)
    finally:
        for x in (ref, b, c):
            x.close()


def test_pair_errors():
    mask, u0, u1 = case()
    g = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
    try:
        with pytest.raises(les.LesError) as e:
            g.set_inflow_pair(0.0, u0, 1.0, u1)
        assert e.value.code == les.LES_ESTATE
        g.set_inflow(u0, 0.01, 3)
        for t0, t1 in ((1.0, 1.0), (2.0, 1.0), (0.0, float("inf"))):
            with pytest.raises(les.LesError) as e:
                g.set_inflow_pair(t0, u0, t1, u1)
            assert e.value.code == les.LES_EINVAL
        bad = u1.copy()
        bad[2] = np.nan
        with pytest.raises(les.LesError):
            g.set_inflow_pair(0.0, u0, 1.0, bad)
    finally:
        g.close()


@pytest.mark.parametrize("mode", [les.ENSEMBLE_BATCHED, les.ENSEMBLE_PERSISTENT])
def test_ensemble_interpolates_like_single_handles(mode):
    """Members with different pairs (and one plain member) stepped as an
    ensemble equal the same handles stepped alone, bit for bit: the
    ensemble forms each member's weight on the device from its step count
    with the same float64 arithmetic as the host."""
    print(f"[ensemble pairs] mode {mode}", flush=True)
    settings = [(3, (1 * DT, 5 * DT)), (4, (0.0, 3 * DT)), (5, None)]
    ens_m, single = [], []
    for seed, pair in settings:
        mask, u0, u1 = case(seed)
        for lst in (ens_m, single):
            x = les.LES(NX, NY, NZ, 4.0, 4.0, 2.0, DT, mask)
            x.set_inflow(u0, 0.01, seed)
            if pair is not None:
                x.set_inflow_pair(pair[0], u0, pair[1], u1 * (1 + 0.1 * seed))
            lst.append(x)
    ens = les.Ensemble(ens_m)
    try:
        ens.set_mode(mode)
        _, _, iters = ens.step(6)
        for q, b in enumerate(single):
            _, _, it_b = b.step(6)
            assert list(iters[:, q]) == list(it_b), q
            for x, y in zip(ens_m[q].get_fields(), b.get_fields()):
                assert np.array_equal(x, y), q
    finally:
        ens.close()
        for x in ens_m + single:
            x.close()


class Replay:
    """The oracle, stepping with the GPU run's iteration counts."""

    def __init__(self, o, iters):
        self.o, self.iters = o, list(iters)

    def set_inflow(self, p, a, s):
        self.o.set_inflow(p, a, s)

    def set_inflow_pair(self, *args):
        self.o.set_inflow_pair(*args)

    def step(self, n):
        return self.o.step(1, forced=[self.iters.pop(0)])


def feed_from_thread(times, profs):
    feed = ProfileFeed()

    def run():
        for t, p in zip(times, profs):
            feed.push(t, p)
        feed.close()

    th = threading.Thread(target=run, daemon=True)
    th.start()
    return feed, th


def test_feed_driven_run_matches_oracle():
    """A producer thread delivers a profile every 4 steps; the coupled loop
    on the GPU and the oracle replaying it end within the parity bar."""
    print("[coupled feed]", flush=True)
    mask, u0, u1 = case(5)
    times = [4 * DT * q for q in range(4)]
    profs = [((1 - q / 3) * u0 + (q / 3) * u1).astype(np.float32) for q in range(4)]
    g, o = make(mask)
    try:
        feed, th = feed_from_thread(times, profs)
        cg = CoupledInflow(g, feed, DT, noise_amp=0.01, seed=5, timeout=30)
        iters = []
        for _ in range(12):
            _, _, it = cg.step()
            iters.append(int(it[0]))
        th.join()
        feed, th = feed_from_thread(times, profs)
        co = CoupledInflow(Replay(o, iters), feed, DT, noise_amp=0.01, seed=5, timeout=30)
        for _ in range(12):
            co.step()
        th.join()
        assert cg.pairs == co.pairs and len(cg.pairs) == 3
        errs = [rel(x, y) for x, y in zip(g.get_fields(), o.get_fields())]
        print(f"  pairs {cg.pairs} fields {max(errs):.2e}", flush=True)
        assert max(errs) <= 1e-4
    finally:
        g.close()

"""Host side of the coupled inflow (section 4, the coupled WRF/LES time loop).

A driving model (WRF in the paper) delivers a wind profile every simulated
minute while the LES steps at half a second.  Before each step the LES
synchronises with the driver, takes the data that has arrived, and
interpolates the profile for its own time between the two latest samples;
it does no model work until two samples exist.

``ProfileFeed`` is the exchange: a FIFO of (time, profile) samples that a
producer thread fills and closes.  ``CoupledInflow`` is the LES side: it
advances a model one step at a time, pulling samples so that the newest is
at or past the step's start time, and hands the two newest to the model's
``set_inflow_pair`` (the interpolation itself runs on the device, inside
the step).  The model is anything with ``set_inflow(profile, noise_amp,
seed)``, ``set_inflow_pair(t0, prof0, t1, prof1)`` and ``step(1)``.
"""
from __future__ import annotations

import queue

import numpy as np

_END = object()


class ProfileFeed:
    """FIFO of inflow profile samples from a driving model.  Times must
    increase strictly; ``close`` marks the end of the run."""

    def __init__(self, maxsize: int = 0):
        self._q: queue.Queue = queue.Queue(maxsize)

    def push(self, t: float, profile) -> None:
        self._q.put((float(t), np.array(profile, dtype=np.float32)))

    def close(self) -> None:
        self._q.put(_END)

    def get(self, timeout: float | None):
        """The next sample, or None once the feed is closed.  Raises
        queue.Empty after `timeout` seconds without one."""
        item = self._q.get(timeout=timeout)
        return None if item is _END else item


class CoupledInflow:
    """Steps `model` with its inflow driven by `feed`.

    Before the step that starts at time n dt (n = steps done) it takes
    samples until the newest is at or after that time, or the feed has
    ended; with fewer than two samples it waits (there is nothing to
    interpolate between yet).  The first sample also sets the initial
    state through ``set_inflow``.  ``pairs`` records (step, t0, t1) each
    time a new pair is handed over."""

    def __init__(self, model, feed: ProfileFeed, dt: float, noise_amp: float = 0.01,
                 seed: int = 0, timeout: float = 60.0):
        if not dt > 0:
            raise ValueError("dt must be positive")
        self.model, self.feed, self.dt = model, feed, float(dt)
        self.noise_amp, self.seed, self.timeout = float(noise_amp), int(seed), timeout
        self.samples: list = []          # the two newest (time, profile)
        self.ended = False
        self.started = False
        self.n = 0
        self.pairs: list = []
        self._pair = None

    def _pull(self) -> None:
        item = self.feed.get(self.timeout)
        if item is None:
            self.ended = True
            return
        t, prof = item
        if self.samples and not t > self.samples[-1][0]:
            raise ValueError(f"sample times must increase ({t} after {self.samples[-1][0]})")
        self.samples = (self.samples + [(t, prof)])[-2:]

    def step(self):
        """One model step; returns what ``model.step(1)`` returns."""
        t = self.n * self.dt
        while not self.ended and (len(self.samples) < 2 or self.samples[-1][0] < t):
            self._pull()
        if len(self.samples) < 2:
            raise RuntimeError("the feed ended before two profile samples arrived")
        (ta, pa), (tb, pb) = self.samples
        if not self.started:
            self.model.set_inflow(pa, self.noise_amp, self.seed)
            self.started = True
        if self._pair != (ta, tb):
            self.model.set_inflow_pair(ta, pa, tb, pb)
            self._pair = (ta, tb)
            self.pairs.append((self.n, ta, tb))
        out = self.model.step(1)
        self.n += 1
        return out

"""CPU tests of the serving mix's input recipe (`meshgen.mixed_stream`): the stated shapes,
sizes, material and frequency ranges and plane-wave counts, the redraw rule (at least 10 mean
edges per interior wavelength), the plane waves' unit directions and transverse polarisations,
and a reproducible stream for a given seed."""
from __future__ import annotations

import math

import numpy as np
import pytest

import meshgen

N = 40


@pytest.fixture(scope="module")
def stream():
    return meshgen.mixed_stream(N, rate_hz=2.0, seed=5)


def test_shapes_sizes_and_ranges(stream):
    kinds = set()
    for _, w in stream:
        kind = w.name.split("_")[0].rstrip("0123456789")
        kinds.add(kind)
        assert kind in ("sphere", "ellipsoid", "cube")
        nt = len(w.tri)
        n = round(math.sqrt(nt / 12))
        assert nt == 12 * n * n
        assert 12 * round(math.sqrt(320 / 12)) ** 2 <= nt <= 12 * round(math.sqrt(20000 / 12)) ** 2
        # circumradius 1 m: sphere vertices on the unit sphere, cube corners at distance 1, the
        # ellipsoid's vertices on x^2 + (y / 0.6)^2 + (z / 0.4)^2 = 1
        r = np.linalg.norm(w.xyz, axis=1)
        if kind == "sphere":
            assert np.allclose(r, 1.0), w.name
        elif kind == "cube":
            assert abs(r.max() - 1.0) < 1e-9, w.name
        else:
            q = (w.xyz / np.array([1.0, 0.6, 0.4])) ** 2
            assert np.allclose(q.sum(axis=1), 1.0), w.name
            assert 0.99 < r.max() <= 1.0 + 1e-12, w.name
        eps = w.eps_r[0]
        k0a = 2 * math.pi * w.freq_hz / meshgen.C0
        assert 1.5 <= eps <= 10.0 and 0.5 <= k0a <= 10.0
        assert 1 <= len(w.khat) <= 64 and w.pol.shape == (len(w.khat), 3)
        # the redraw rule: at least 10 mean edges per interior wavelength
        h = meshgen.mean_edge(w.xyz, w.tri)
        assert 2 * math.pi / (k0a * math.sqrt(eps)) / h >= 10.0, w.name
        # unit directions, polarisations transverse to them
        assert np.allclose(np.linalg.norm(w.khat, axis=1), 1.0)
        assert np.allclose(np.einsum("ij,ij->i", w.khat, w.pol.real), 0.0, atol=1e-12)
    assert kinds == {"sphere", "ellipsoid", "cube"}


def test_arrivals_and_reproducibility(stream):
    times = np.array([t for t, _ in stream])
    assert np.all(np.diff(times) > 0)
    # Poisson arrivals at 2 per second: the mean gap of 40 draws is within 3 standard errors
    assert abs(np.diff(np.concatenate([[0.0], times])).mean() - 0.5) < 3 * 0.5 / math.sqrt(N)
    again = meshgen.mixed_stream(8, rate_hz=2.0, seed=5)
    assert [w.name for _, w in again] == [w.name for _, w in stream[:8]]
    assert [t for t, _ in again] == list(times[:8])
    other = meshgen.mixed_stream(8, rate_hz=2.0, seed=6)
    assert [w.name for _, w in other] != [w.name for _, w in stream[:8]]

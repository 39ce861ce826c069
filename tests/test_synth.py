"""Seeded input generators: determinism and basic statistics."""
import hashlib

import numpy as np

import synth


def digest(cat):
    h = hashlib.sha256()
    for a in cat.arrays():
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_uniform_deterministic():
    a = synth.uniform_catalogue(0, 500, 60.0)
    b = synth.uniform_catalogue(0, 500, 60.0)
    c = synth.uniform_catalogue(1, 500, 60.0)
    assert digest(a) == digest(b) != digest(c)
    assert a.x.min() >= 0 and a.x.max() < 60 and a.w.min() >= 0.5 and a.w.max() < 1.5


def test_grf_deterministic_and_scaled():
    a = synth.grf_catalogue(3, 2000, 100.0, ngrid=256)
    b = synth.grf_catalogue(3, 2000, 100.0, ngrid=256)
    assert digest(a) == digest(b)
    rng = np.random.default_rng(0)
    kappa, gamma = synth.grf_fields(rng, 256, 100.0, sigma=0.02)
    assert abs(kappa.std() - 0.02) < 1e-12
    # Kaiser-Squires has unit modulus away from l = 0: shear power = kappa power
    assert abs(np.mean(np.abs(gamma) ** 2) / np.mean(kappa ** 2) - 1.0) < 1e-10


def test_lognormal_exact_count():
    c = synth.lognormal_catalogue(4, 5000, 100.0, ngrid=128)
    assert c.n == 5000
    assert c.x.min() >= 0 and c.x.max() <= 100.0


def test_log_edges():
    e = synth.log_edges(1.0, 30.0, 4)
    assert e[0] == 1.0 and e[-1] == 30.0
    assert np.allclose(np.diff(np.log(e)), np.log(30.0) / 4)


def test_serving_stream_params():
    reqs = synth.serving_requests(16)
    assert len(reqs) == 16
    for r in reqs:
        assert 8 <= r["nbins"] <= 16 and r["nmax"] == 8
        assert 1e5 <= r["n"] <= 2e6 + 1

"""Serving on the GPU: every request's result in a concurrent mix equals its
result served alone (bit for bit: the tile decomposition is the same and no
reduction depends on timing), equals a direct estimate, and matches the FP64
oracle; admission never exceeds the HBM budget; a failing or cancelled
request leaves the others intact."""
import numpy as np
import pytest

import oracle
import synth
from helpers import rel_per_mu

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp16": 1e-5, "bf16": 1e-5}


@pytest.fixture(scope="module")
def fp():
    import paper_2509_07974_amd as m
    m.lib()
    return m


def make_jobs():
    from paper_2509_07974_amd.serve import Job
    specs = [  # (n, side, nbins, nmax, precision)
        (300, 30.0, 3, 3, "fp64"),
        (1500, 50.0, 5, 4, "fp16"),
        (800, 40.0, 4, 3, "bf16"),
        (2500, 60.0, 4, 4, "fp16"),
        (600, 35.0, 3, 2, "fp64"),
        (1200, 45.0, 5, 3, "fp16"),
    ]
    jobs = []
    for r, (n, side, nb, nmax, prec) in enumerate(specs):
        cat = synth.uniform_catalogue(500 + r, n, side)
        jobs.append(Job(r, *cat.arrays(), synth.log_edges(1.0, 20.0, nb), nmax, precision=prec))
    return jobs


def serve(jobs, **kw):
    from paper_2509_07974_amd.serve import Server
    srv = Server(**kw)
    for j in jobs:
        srv.submit(j)
    srv.drain()
    return srv


def test_mix_equals_alone_and_direct_and_oracle(fp):
    mix = make_jobs()
    srv = serve(mix, tile_centers=256, inflight=3)
    assert all(j.state == "done" for j in mix), [(j.rid, j.state, j.error) for j in mix]
    assert srv.used == 0
    for j in make_jobs():
        alone = serve([j], tile_centers=256)
        assert j.state == "done"
        m = mix[j.rid]
        assert m.ntiles == j.ntiles and m.ntiles >= 2
        assert np.array_equal(m.result, j.result), j.rid
        direct = fp.estimate_4pcf_multipoles(j.x, j.y, j.g1, j.g2, j.w, j.edges, j.nmax,
                                             precision=j.precision, tile_centers=j.tile_centers)
        assert np.array_equal(direct, j.result), j.rid
        del alone
    for r in (0, 2, 4):
        j = mix[r]
        ref = oracle.upsilon(j.x, j.y, j.g1, j.g2, j.w, j.edges, j.nmax)
        assert np.all(rel_per_mu(j.result, ref) < TOL[j.precision]), (r, rel_per_mu(j.result, ref))


def test_admission_respects_budget(fp):
    jobs = make_jobs()
    from paper_2509_07974_amd import plan
    fps = [plan(j.n, j.edges, j.nmax, j.precision, tile_centers=256)[0] for j in jobs]
    budget = int(2.2 * max(fps))
    srv = serve(jobs, tile_centers=256, hbm_budget=budget)
    assert all(j.state == "done" for j in jobs)
    assert srv.peak_used <= budget
    assert srv.peak_used >= max(fps)


def test_failure_and_cancellation_isolated(fp):
    from paper_2509_07974_amd.serve import Server
    jobs = make_jobs()
    jobs[1].x = jobs[1].x.copy()
    jobs[1].x[7] = np.nan
    srv = Server(tile_centers=256)
    for j in jobs:
        srv.submit(j)
    srv.cancel(3)
    srv.drain()
    st = {j.rid: j.state for j in jobs}
    assert st[1] == "failed" and jobs[1].error.status == -1
    assert st[3] == "cancelled"
    for r in (0, 2, 4, 5):
        assert st[r] == "done"
    ref = make_jobs()
    for r in (0, 5):
        alone = serve([ref[r]], tile_centers=256)
        assert np.array_equal(ref[r].result, jobs[r].result)
        del alone
    assert srv.used == 0

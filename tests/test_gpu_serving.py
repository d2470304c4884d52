"""Serving loop: continuous batching with segmented launches.

A result must not depend on what else runs: each request solved in a mix of
requests of other sizes, densities and precisions gives the same generators
and energy as solved alone by scvt_solve (bitwise here; the stated tolerance
is 1e-12 relative), and a served FP64 request follows the oracle's
trajectory."""
import math

import numpy as np
import pytest

import paper_1709_06924_amd.inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scvt():
    from paper_1709_06924_amd import scvt as mod
    return mod


def make_requests():
    stream = I.serving_stream(seed=4, rate=20.0, count=6, n_lo=3000, n_hi=40000)
    return [(I.uniform_sphere(r["n"], r["z0_seed"]), r["density"]) for r in stream]


def serve_all(scvt, reqs, tol, cap, max_slots, **common):
    srv = scvt.Server(16 << 30, max_slots=max_slots)
    ids = [srv.submit(z, d, tol, cap, **dict(common, **kw)) for z, d, kw in reqs]
    out = {}
    while len(out) < len(ids):
        for rid in ids:
            if rid not in out:
                res = srv.poll(rid)
                if res is not None:
                    out[rid] = res
    srv.close()
    return [out[r] for r in ids]


def test_batch_invariance_alone_vs_mix(scvt):
    """Six requests of the serving stream's kind (mixed precision, tanh
    densities) served four at a time, against scvt_solve of each alone."""
    reqs = [(z, d, {}) for z, d in make_requests()]
    tol, cap = 1e-8, 25
    served = serve_all(scvt, reqs, tol, cap, 4, precision="mixed", m_hist=10)
    for res, (z0, d, _) in zip(served, reqs):
        S = scvt.Solver(z0, d, precision="mixed", m_hist=10)
        S.solve(cap, tol)
        alone_z = S.generators()
        alone_F = S.energy()[0]
        assert res["status"] >= 0
        assert res["info"]["iter"] == S.info.iter
        assert res["info"]["n_evals"] == S.info.n_evals
        assert np.max(np.abs(res["z"] - alone_z)) <= 1e-12
        assert abs(res["info"]["F"] - alone_F) <= 1e-12 * alone_F
        assert np.array_equal(res["z"], alone_z)   # bitwise in practice
        S.close()


def test_segmented_mix_of_kinds(scvt):
    """One round batches requests with different cell paths (n = 200: every
    cell by the fallback clipper), vector widths (3n odd), precisions and
    density variants (one quadrature launch per variant): each result is
    bit-identical to its scvt_solve alone."""
    reqs = [(I.uniform_sphere(200, 51), I.density_tanh(I.latlon(10, 20), 0.6, 0.3, 4), {}),
            (I.uniform_sphere(3001, 52), {"kind": "const"}, {"precision": "fp64"}),
            (I.uniform_sphere(10007, 53), I.density_two_centre(), {"precision": "fp64"}),
            (I.uniform_sphere(20000, 54), I.density_x3(), {"precision": "mixed"}),
            (I.uniform_sphere(8000, 55), I.density_tanh(I.latlon(-40, 70), 0.5, 0.15, 16),
             {"precision": "mixed", "m_hist": 3})]
    tol, cap = 1e-9, 15
    served = serve_all(scvt, reqs, tol, cap, 8, m_hist=7)
    for res, (z0, d, kw) in zip(served, reqs):
        kw = dict({"m_hist": 7}, **kw)
        S = scvt.Solver(z0, d, **kw)
        S.solve(cap, tol)
        assert res["status"] >= 0, res["status"]
        assert res["info"]["iter"] == S.info.iter and res["info"]["n_evals"] == S.info.n_evals
        assert np.array_equal(res["z"], S.generators())
        assert res["info"]["F"] == S.energy()[0]
        S.close()


def test_served_request_follows_the_oracle(scvt):
    """An FP64 request served among others: its 8 iterations match the
    oracle's P-LBFGS trajectory (the trajectory tolerance of the parity
    tests)."""
    import oracle
    d = I.density_tanh(I.latlon(30, 90), math.pi / 6, 0.2, 8)
    z0 = I.uniform_sphere(2562, 61)
    reqs = [(z0, d, {"precision": "fp64"}),
            (I.uniform_sphere(5000, 62), d, {"precision": "mixed"}),
            (I.uniform_sphere(900, 63), {"kind": "const"}, {"precision": "fp64"})]
    served = serve_all(scvt, reqs, 0.0, 8, 4, m_hist=7)
    res = served[0]
    S = scvt.Solver(z0, d, m_hist=7)  # the library's renormalised rows
    O = oracle.Solver(S.generators(), d, m_hist=7)
    S.close()
    for _ in range(8):
        O.step()
    assert res["status"] == 1 and res["info"]["iter"] == 8  # stopped at the cap
    assert res["info"]["n_evals"] == O.n_evals
    assert np.max(np.abs(res["z"] - O.Z)) < 1e-10
    assert abs(res["info"]["F"] - O.cur.F) <= 1e-10 * O.cur.F


def test_admission_by_footprint(scvt):
    reqs = make_requests()
    fps = [scvt.footprint(len(z), d, m_hist=10, precision="mixed") for z, d in reqs]
    budget = sorted(fps)[-1] + sorted(fps)[-2] + 1   # at most two of the largest fit
    srv = scvt.Server(budget, max_slots=8)
    ids = [srv.submit(z, d, 1e-8, 10, precision="mixed", m_hist=10) for z, d in reqs]
    done = set()
    peak = 0
    while len(done) < len(ids):
        st = srv.stats()
        assert st["bytes_used"] <= budget
        peak = max(peak, st["running"])
        for rid in ids:
            if rid not in done and srv.poll(rid, want_z=False) is not None:
                done.add(rid)
    srv.close()
    assert peak >= 1


def test_oversized_request_rejected(scvt):
    z = I.uniform_sphere(20000, 1)
    fp = scvt.footprint(20000, {"kind": "const"}, m_hist=10)
    srv = scvt.Server(fp // 2, max_slots=2)
    with pytest.raises(scvt.ScvtError) as e:
        srv.submit(z, {"kind": "const"}, 1e-8, 10, m_hist=10)
    assert e.value.code == -2
    srv.close()


def test_poisson_stream_latency(scvt):
    from paper_1709_06924_amd import serving
    stream = I.serving_stream(seed=4, rate=40.0, count=8, n_lo=2000, n_hi=20000)
    records, summary = serving.run_stream(stream, tol=1e-8, max_iter=30, max_slots=4,
                                          hbm_budget=16 << 30)
    print(summary)
    assert summary["requests"] == 8 and summary["failed"] == 0
    assert summary["p99_s"] >= summary["p50_s"] > 0

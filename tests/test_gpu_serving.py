"""Request server (lspr_server_*): continuous batching of mixed requests on one GPU.

What is checked: a request's results are the same alone and in a mix of concurrent requests
(every kernel sums in a fixed order, so the bar is equality up to 1e-12 relative on C_ext,
far inside the 1e-4 FP32 tolerance), the mix really overlaps on the device, the admission
estimate bounds every request's measured peak of device memory, the budget is never
over-reserved, failures stay with their own request, and a small multi-surface request matches
the oracle, with and without point charges in an analyte.
"""
import numpy as np
import pytest

import oracle
from lspr_inputs import (octasphere, perturbed_ellipsoid, place_at_gap, merge_surfaces,
                         eps_silver_drude, wavelength_grid, EPS_WATER)

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1812_10722_amd import lspr
    assert torch.cuda.is_available()
    return lspr


def _request(k, nu, n_blobs, nu_blob, n_lambda, seed=11):
    """A seeded request: sphere R = 10 nm plus blobs at 0.5-3 nm gaps, lambdas in 350-420."""
    rng = np.random.default_rng([seed, k])
    surfs = [octasphere(nu, 10.0)]
    for b in range(n_blobs):
        bv, bt = perturbed_ellipsoid(nu_blob, (2.0, 7.0, 2.0), rng)
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        # spread the blobs around the sphere so they cannot overlap
        d = d + 2.5 * np.eye(3)[b % 3] * (1 if b < 3 else -1)
        d /= np.linalg.norm(d)
        surfs.append((place_at_gap(bv, d, 10.0, rng.uniform(0.5, 3.0)), bt))
    lam = np.sort(rng.uniform(350.0, 420.0, n_lambda))
    em = np.full(n_lambda, EPS_WATER + 0j)
    es = np.concatenate([eps_silver_drude(lam)[:, None],
                         np.full((n_lambda, n_blobs), 2.5 + 0j)], 1)
    return surfs, lam, em, es


MIX = [(0, 24, 0, 0, 16), (1, 40, 2, 20, 8), (2, 16, 1, 16, 33), (3, 32, 3, 18, 5),
       (4, 20, 0, 0, 64), (5, 28, 1, 24, 12)]


def _op(lib):
    return lib.op_params(k_far=4, k_fine=19, n_k=9, method="treecode", p=8, theta=0.5,
                         precision="fp32")


def _gm(lib):
    return lib.gmres_params(tol=1e-6, restart=60, max_iter=600)


def _run(lib, reqs, max_slots, budget=0):
    sv = lib.Server(hbm_budget_bytes=budget, max_slots=max_slots)
    try:
        tickets = [sv.submit(s, lam, em, es, op=_op(lib), gmres=_gm(lib))
                   for s, lam, em, es in reqs]
        out = [sv.poll(t, wait=True) for t in tickets]
        return out, sv.stats()
    finally:
        sv.close()


@pytest.fixture(scope="module")
def mix_requests():
    return [_request(*m) for m in MIX]


@pytest.fixture(scope="module")
def alone_results(lib, mix_requests):
    res = []
    for r in mix_requests:
        out, st = _run(lib, [r], 1)
        assert st["max_active"] == 1
        res.append(out[0])
    return res


def test_alone_equals_mix(lib, mix_requests, alone_results):
    mix, st = _run(lib, mix_requests, 4)
    assert st["completed"] == len(MIX)
    assert st["max_active"] >= 2, st  # requests were on the device together
    for k, (a, m) in enumerate(zip(alone_results, mix)):
        assert a["status"] == lib.LSPR_OK and m["status"] == lib.LSPR_OK, (k, a["error"], m["error"])
        for key in ("cext_sensor", "cext_total"):
            rel = np.abs(m[key] - a[key]) / np.abs(a[key])
            assert rel.max() <= 1e-12, (k, key, rel.max())
        assert np.array_equal(a["iters"], m["iters"]), k


def test_server_matches_geometry_api(lib, mix_requests, alone_results):
    """The server runs the same path as lspr_geometry_create + lspr_solve."""
    surfs, lam, em, es = mix_requests[1]
    geo = lib.Geometry(surfs, op=_op(lib))
    r = geo.solve(lam, em, es, gmres=_gm(lib))
    geo.close()
    rel = np.abs(r["cext_sensor"] - alone_results[1]["cext_sensor"]) / np.abs(r["cext_sensor"])
    assert rel.max() <= 1e-12, rel.max()


def test_footprint_bounds_measured_peak(lib, mix_requests, alone_results):
    for k, a in enumerate(alone_results):
        assert 0 < a["peak_bytes"] <= a["est_bytes"], (k, a["peak_bytes"], a["est_bytes"])
        # and the estimate is not wildly loose for these sizes
        assert a["est_bytes"] <= 12 * a["peak_bytes"] + (256 << 20), (k, a["est_bytes"], a["peak_bytes"])
        n = sum(len(t) for _, t in mix_requests[k][0])
        assert a["est_bytes"] == lib.lspr_request_footprint(
            n, len(mix_requests[k][0]), len(mix_requests[k][1]), _op(lib), _gm(lib))


def test_budget_is_never_over_reserved(lib, mix_requests):
    reqs = mix_requests[:4]
    ests = [lib.lspr_request_footprint(sum(len(t) for _, t in s), len(s), len(lam), _op(lib),
                                       _gm(lib)) for s, lam, _, _ in reqs]
    budget = int(1.2 * max(ests))
    out, st = _run(lib, reqs, 4, budget=budget)
    assert st["budget_bytes"] == budget
    assert st["peak_reserved_bytes"] <= budget
    assert st["estimate_violations"] == 0
    assert all(o["status"] == lib.LSPR_OK for o in out)
    # admission order is arrival order
    admits = [o["t_admit"] for o in out]
    assert admits == sorted(admits)


def test_oversize_request_is_rejected(lib, mix_requests):
    sv = lib.Server(hbm_budget_bytes=1 << 20, max_slots=2)
    try:
        s, lam, em, es = mix_requests[0]
        with pytest.raises(lib.LsprError) as e:
            sv.submit(s, lam, em, es, op=_op(lib), gmres=_gm(lib))
        assert e.value.code == lib.LSPR_E_NOMEM
    finally:
        sv.close()


def test_failure_stays_with_its_request(lib, mix_requests):
    good = mix_requests[0]
    v, t = octasphere(12, 10.0)
    bad = ([(v, t[:-1])], good[1], good[2], good[3][:, :1])  # open surface
    sv = lib.Server(max_slots=2)
    try:
        tb = sv.submit(*bad, op=_op(lib), gmres=_gm(lib))
        tg = sv.submit(*good, op=_op(lib), gmres=_gm(lib))
        rb = sv.poll(tb, wait=True)
        rg = sv.poll(tg, wait=True)
    finally:
        sv.close()
    assert rb["status"] == lib.LSPR_E_MESH and "open surface" in rb["error"]
    assert rg["status"] == lib.LSPR_OK


def test_poll_busy_then_done(lib, mix_requests):
    s, lam, em, es = mix_requests[4]
    sv = lib.Server(max_slots=1)
    try:
        t = sv.submit(s, lam, em, es, op=_op(lib), gmres=_gm(lib))
        first = sv.poll(t, wait=False)  # usually still running: None
        r = first if first is not None else sv.poll(t, wait=True)
        assert r["status"] == lib.LSPR_OK and r["latency_s"] > 0
        with pytest.raises(lib.LsprError):
            sv.poll(t, wait=True)  # ticket released
    finally:
        sv.close()


def test_small_multi_surface_request_matches_oracle(lib):
    """A served request with two analytes against the dense FP64 oracle (FP32 bar 1e-4)."""
    rng = np.random.default_rng(21)
    s = octasphere(8, 8.0)
    bv, bt = perturbed_ellipsoid(5, (1.5, 4.0, 1.5), rng)
    surfs = [s, (place_at_gap(bv, [0, 0, 1.0], 8.0, 1.0), bt),
             (place_at_gap(bv, [0, 0, -1.0], 8.0, 1.0), bt)]
    lam = wavelength_grid(375.0, 395.0, 5)
    em = np.full(5, EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(5, 2.5 + 0j), np.full(5, 2.5 + 0j)], 1)
    sv = lib.Server(max_slots=2)
    try:
        r = sv.poll(sv.submit(surfs, lam, em, es, op=_op(lib),
                              gmres=lib.gmres_params(tol=1e-6)), wait=True)
    finally:
        sv.close()
    v, t, sid = merge_surfaces(surfs)
    ref = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
    for key in ("cext_sensor", "cext_total"):
        rel = np.abs(r[key] - ref[key]) / np.abs(ref[key])
        assert rel.max() < 1e-4, (key, rel.max())


def test_request_with_charges_matches_oracle(lib):
    """Point charges inside one analyte of a served request (Eq. integral_eq_lspr_system, last
    row) against the dense FP64 oracle with the same charges (FP32 bar 1e-4); the charges move
    C_ext by far more than that, and a charge outside the listed surfaces fails the submit."""
    rng = np.random.default_rng(23)
    s = octasphere(8, 8.0)
    bv, bt = perturbed_ellipsoid(5, (1.5, 4.0, 1.5), rng)
    blob = place_at_gap(bv, [0, 0, 1.0], 8.0, 1.0)
    surfs = [s, (blob, bt)]
    pos = blob.mean(0)[None, :] + 0.3 * rng.standard_normal((2, 3))
    charges = (pos, np.array([2 * 18.0951, -18.0951]), np.array([1, 1]))  # +2 e, -1 e
    lam = wavelength_grid(378.0, 392.0, 4)
    em = np.full(4, EPS_WATER + 0j)
    es = np.stack([eps_silver_drude(lam), np.full(4, 2.5 + 0.1j)], 1)
    sv = lib.Server(max_slots=2)
    try:
        with pytest.raises(lib.LsprError):
            sv.submit(surfs, lam, em, es, op=_op(lib), charges=(pos, [1.0, 1.0], [1, 2]))
        # FP32 products: tol 1e-6 (1e-7 is near what they can resolve), as the geometry test
        r = sv.poll(sv.submit(surfs, lam, em, es, op=_op(lib),
                              gmres=lib.gmres_params(tol=1e-6, restart=100, max_iter=1000),
                              charges=charges), wait=True)
    finally:
        sv.close()
    assert r["status"] == 0, r["error"]
    v, t, sid = merge_surfaces(surfs)
    ref = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19, charges=charges)
    ref0 = oracle.solve(v, t, sid, lam, em, es, [0, 0, 1.0], k_far=4, k_fine=19)
    for key in ("cext_sensor", "cext_total"):
        rel = np.abs(r[key] - ref[key]) / np.abs(ref[key])
        assert rel.max() < 1e-4, (key, rel.max())
    assert (np.abs(ref0["cext_total"] / ref["cext_total"] - 1)).max() > 1e-3


def test_burst_of_large_requests_all_succeed(lib):
    """The first 12 requests of the seeded serving stream (16400-258080 panels) submitted at
    once on 4 slots: the reservations come close to the budget, so memory freed by finished
    requests must be reusable or returned by the pool (a regression: it once ran the device out
    of memory while the reservations still fitted)."""
    from lspr_inputs import serving_stream
    reqs = [w for _, w in serving_stream(seed=5, n_requests=12)]
    sv = lib.Server(max_slots=4)
    try:
        tickets = [sv.submit(w.surfaces, w.lambdas, w.eps_medium, w.eps_surface, w.e_field,
                             op=lib.op_params(**w.op), gmres=lib.gmres_params(**w.gmres))
                   for w in reqs]
        out = [sv.poll(t, wait=True) for t in tickets]
        st = sv.stats()
    finally:
        sv.close()
    assert all(r["status"] == lib.LSPR_OK for r in out), [(r["status"], r["error"]) for r in out]
    assert st["estimate_violations"] == 0
    assert all(0 < r["peak_bytes"] <= r["est_bytes"] for r in out)

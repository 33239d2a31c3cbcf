"""Synthetic input generators: closed, consistently oriented meshes of the stated sizes."""
import numpy as np
import pytest

from lspr_inputs import (octasphere, perturbed_ellipsoid, place_at_gap, eps_silver_drude,
                         wavelength_grid, workload, serving_stream)


def _check_closed_oriented(v, t):
    # every directed edge appears once and its reverse appears once: closed, 2-manifold,
    # consistently oriented
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    fwd = {tuple(x) for x in e.tolist()}
    assert len(fwd) == len(e)
    assert all((b, a) in fwd for a, b in fwd)
    a = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    vol = np.sum(np.einsum("ij,ij->i", a, v[t].mean(1))) / 6.0
    assert vol > 0
    assert np.linalg.norm(a, axis=1).min() > 0
    return vol


@pytest.mark.parametrize("nu", [1, 3, 8, 16])
def test_octasphere_counts_and_topology(nu):
    v, t = octasphere(nu, 2.5)
    assert len(t) == 8 * nu * nu and len(v) == 4 * nu * nu + 2
    assert np.allclose(np.linalg.norm(v, axis=1), 2.5)
    _check_closed_oriented(v, t)


def test_perturbed_ellipsoid_and_gap():
    rng = np.random.default_rng(0)
    v, t = perturbed_ellipsoid(12, (2.0, 7.0, 2.0), rng)
    vol = _check_closed_oriented(v, t)
    assert 0.7 < vol / (4 / 3 * np.pi * 28.0) < 1.3
    p = place_at_gap(v, [0, 0, 1.0], 8.0, 1.0)
    assert abs(np.min(np.linalg.norm(p, axis=1)) - 9.0) < 1e-9
    # same seed, same blob
    v2, _ = perturbed_ellipsoid(12, (2.0, 7.0, 2.0), np.random.default_rng(0))
    assert np.array_equal(v, v2)


def test_drude_matches_paper_silver_at_380nm():
    """The Drude parameters reproduce the paper's eps_Ag(380 nm) = -3.3877 + 0.1922i."""
    e = eps_silver_drude(380.0)
    assert abs(e.real + 3.3877) < 5e-4 and abs(e.imag - 0.1922) < 5e-4
    lam = wavelength_grid(350, 420, 64)
    assert lam[0] == 350 and lam[-1] == 420 and len(lam) == 64


def test_workload_shapes():
    w1 = workload("sphere_512")
    assert w1.n_panels == 512 and w1.eps_surface.shape == (1, 1)
    w2 = workload("sphere_32k_sweep")
    assert w2.n_panels == 32768 and len(w2.lambdas) == 64
    w3 = workload("sensor_two_analytes")
    assert [len(t) for _, t in w3.surfaces] == [40328, 29768, 29768]
    assert w3.eps_surface.shape == (32, 3)
    for v, t in w3.surfaces[1:]:
        assert abs(np.min(np.linalg.norm(v, axis=1)) - 9.0) < 1e-9   # 1 nm gap to R = 8


def test_serving_stream_is_seeded():
    a = [(t, w.n_panels, len(w.lambdas)) for t, w in
         zip(range(3), (x for _, x in serving_stream(n_requests=3, nu_range=(16, 20),
                                                     blob_nu_range=(8, 10))))]
    b = [(t, w.n_panels, len(w.lambdas)) for t, w in
         zip(range(3), (x for _, x in serving_stream(n_requests=3, nu_range=(16, 20),
                                                     blob_nu_range=(8, 10))))]
    assert a == b

"""lspr_apply_noalloc (the product for callers that cannot allocate) against lspr_apply: the
same kernels in the same order on a fixed scratch array, so the results must be identical.
Two calls in a row, the second on a smaller geometry with fewer columns (the array keeps the
first call's contents), and a request larger than the array is refused with a clear error."""
import numpy as np
import pytest

from lspr_inputs import octasphere, perturbed_ellipsoid, place_at_gap

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_1812_10722_amd import lspr
    assert torch.cuda.is_available()
    return lspr


def _case(lib, surfs, ncol, seed, **kw):
    rng = np.random.default_rng(seed)
    n = sum(len(t) for _, t in surfs)
    x = rng.standard_normal((ncol, 2 * n)) + 1j * rng.standard_normal((ncol, 2 * n))
    em = np.full(ncol, 1.7733) + 0.01j * rng.standard_normal(ncol)
    es = np.stack([-3.0 + 0.3j + rng.standard_normal(ncol)] +
                  [np.full(ncol, 2.5 + 0.1j)] * (len(surfs) - 1), 1)
    geo = lib.Geometry(surfs, **kw)
    return geo, torch.as_tensor(x).cuda(), em, es


def _compare(lib, geo, xt, em, es):
    ref = geo.apply(xt, em, es).cpu().numpy()
    out = torch.empty_like(xt)
    got = geo.apply(xt, em, es, out=out, noalloc=True).cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale, np.abs(got - ref).max() / scale
    return np.abs(got - ref).max() / scale


def test_noalloc_product_equals_apply_twice_then_smaller(lib):
    rng = np.random.default_rng(4)
    bv, bt = perturbed_ellipsoid(8, (1.5, 4.0, 1.5), rng)
    big = [octasphere(24, 8.0), (place_at_gap(bv, [0, 0, 1.0], 8.0, 0.8), bt)]
    small = [octasphere(8, 10.0)]
    # FP32 treecode products with moments and partial moments (the largest piece list)
    g1, x1, em1, es1 = _case(lib, big, 12, 1, method="treecode", precision="fp32", p=8,
                             theta=0.5)
    # FP64 dense products on a smaller mesh, fewer columns
    g2, x2, em2, es2 = _case(lib, small, 3, 2, method="dense", precision="fp64")
    try:
        e1 = _compare(lib, g1, x1, em1, es1)
        e2 = _compare(lib, g2, x2, em2, es2)
        e3 = _compare(lib, g1, x1[:5].contiguous(), em1[:5], es1[:5])  # big geometry again
        print(f"noalloc vs apply: {e1:.1e} {e2:.1e} {e3:.1e}")
    finally:
        g1.close()
        g2.close()


def test_noalloc_refuses_what_does_not_fit(lib):
    """A product whose temporaries exceed the fixed array fails up front (no launch) with the
    number of bytes it would need; the ordinary entry point still serves it."""
    v, t = octasphere(64, 10.0)  # 32768 panels
    geo = lib.Geometry([(v, t)], method="treecode", precision="fp64", p=8, theta=0.5)
    try:
        n = 2 * len(t)
        x = torch.zeros((64, n), dtype=torch.complex128, device="cuda")
        em = np.full(64, 1.7733 + 0j)
        es = np.full((64, 1), -3.0 + 0.3j)
        with pytest.raises(lib.LsprError) as e:
            geo.apply(x, em, es, noalloc=True)
        assert e.value.code == lib.LSPR_E_INVALID
        assert "bytes of scratch" in str(e.value)
        assert torch.isfinite(geo.apply(x, em, es).abs()).all()
    finally:
        geo.close()

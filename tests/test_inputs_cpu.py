"""The synthetic workload generators: shapes, periodic faces, stability."""
import numpy as np
import pytest

from paper_1507_01265_amd import inputs


def _outflow_over_h(f):
    out = (np.maximum(f.u1[..., 1:], 0) - np.minimum(f.u1[..., :-1], 0)
           + np.maximum(f.u2[:, 1:, :], 0) - np.minimum(f.u2[:, :-1, :], 0)
           + np.maximum(f.u3[1:], 0) - np.minimum(f.u3[:-1], 0))
    return (out / f.h).max()


def _divergence(f):
    return ((f.u1[..., 1:] - f.u1[..., :-1]) + (f.u2[:, 1:, :] - f.u2[:, :-1, :])
            + (f.u3[1:] - f.u3[:-1]))


@pytest.mark.parametrize("make", [inputs.rotation, inputs.divergent_rotation])
def test_rotation_grids_are_periodic_and_stable(make):
    f = make(shape=(16, 64, 128))
    nz, ny, nx = f.psi.shape
    assert f.u1.shape == (nz, ny, nx + 1) and f.u2.shape == (nz, ny + 1, nx)
    assert f.u3.shape == (nz + 1, ny, nx)
    np.testing.assert_array_equal(f.u1[..., nx], f.u1[..., 0])
    np.testing.assert_array_equal(f.u2[:, ny, :], f.u2[:, 0, :])
    np.testing.assert_array_equal(f.u3[nz], f.u3[0])
    assert _outflow_over_h(f) < 1.0
    assert f.psi.min() >= 0.0 and f.psi.max() == 1.0


def test_divergent_rotation_is_divergent_and_rotation_is_not():
    assert np.abs(_divergence(inputs.rotation(shape=(8, 32, 64)))).max() == 0.0
    d = _divergence(inputs.divergent_rotation(shape=(8, 32, 64)))
    assert np.abs(d).max() > 1e-3

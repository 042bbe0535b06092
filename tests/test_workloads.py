"""The seeded generators produce the geometries the benchmarks describe (CPU only)."""
import math

import numpy as np
import pytest

from paper_1602_05650_amd import workloads as W


def test_cgl_nodes_and_fiber_layout():
    a = W.cgl_alpha(31)
    assert a.shape == (32,) and a[0] == 1.0 and a[-1] == -1.0
    assert np.all(np.diff(a) < 0)
    c = W.config0()
    fs = c["fibers"]
    assert fs.n == 512 and fs.n_fib == 16 and fs.nodes_per_fiber == 32
    assert np.all(np.diff(fs.fiber) >= 0)
    x = fs.xyz.reshape(3, 16, 32)
    seg = np.linalg.norm(x[:, :, 0] - x[:, :, -1], axis=0)     # plus end to minus end
    np.testing.assert_allclose(seg, fs.length, rtol=1e-12)
    t = fs.tangent.reshape(3, 16, 32)[:, :, 0]
    np.testing.assert_allclose((x[:, :, 0] - x[:, :, -1]) / seg, t, atol=1e-12)
    centers = x.mean(axis=2)
    assert np.all(np.linalg.norm(centers, axis=0) <= 3.0 + 1e-12)
    assert c["force"].shape == (3, 512)


def test_determinism():
    a, b = W.config0(), W.config0()
    np.testing.assert_array_equal(a["fibers"].xyz, b["fibers"].xyz)
    np.testing.assert_array_equal(a["force"], b["force"])
    r1, r2 = W.serving_request(3, 17), W.serving_request(3, 17)
    np.testing.assert_array_equal(r1["rhs"], r2["rhs"])
    assert r1["iters"] == r2["iters"]
    assert not np.array_equal(W.serving_request(3, 18)["rhs"][:, :5], r1["rhs"][:, :5])


def test_sphere_quadrature():
    R = 5.0
    sph = W.sphere_surface(64, 96, R)
    assert sph.n == 6144
    assert abs(sph.weight.sum() - 4 * math.pi * R * R) < 1e-10 * R * R
    np.testing.assert_allclose(np.linalg.norm(sph.normal, axis=0), 1.0, atol=1e-14)
    np.testing.assert_allclose(sph.xyz, R * sph.normal, atol=1e-13)
    # patch ordering: every run of 32 points is compact
    ext = [np.ptp(sph.xyz[:, k:k + 32], axis=1).max() for k in range(0, sph.n, 32)]
    assert max(ext) < 0.7 * R
    # integrates z^2 exactly: 4 pi R^4 / 3
    assert abs(np.dot(sph.weight, sph.xyz[2] ** 2) - 4 * math.pi * R ** 4 / 3) < 1e-9 * R ** 4


def test_config1_constraints():
    c = W.config1()
    fs = c["fibers"]
    assert fs.n == 32768 and c["sphere"].n == 6144
    r = np.linalg.norm(fs.xyz, axis=0)
    assert r.max() <= 5.0 - 0.05 + 1e-9
    from scipy.spatial import cKDTree
    pairs = cKDTree(fs.xyz.T).query_pairs(0.05, output_type="ndarray")
    assert np.all(fs.fiber[pairs[:, 0]] == fs.fiber[pairs[:, 1]])


@pytest.mark.slow
def test_config2_spindle():
    c = W.config2()
    fs = c["fibers"]
    assert fs.n == 262144 and fs.n_fib == 4096 and fs.nodes_per_fiber == 64
    assert fs.length.min() >= 1.0 and fs.length.max() <= 6.0
    x = fs.xyz.reshape(3, 4096, 64)
    minus = x[:, :, -1]
    pole = np.where(np.arange(4096) < 2048, 4.0, -4.0)
    d = np.linalg.norm(minus - np.stack([pole, 0 * pole, 0 * pole]), axis=0)
    np.testing.assert_allclose(d, 0.5, atol=1e-12)
    t = fs.tangent.reshape(3, 4096, 64)[:, :, 0]
    cosang = -np.sign(pole) * t[0]          # angle to the axis toward the other pole
    assert cosang.min() >= math.cos(math.radians(30.0)) - 1e-12
    np.testing.assert_allclose(c["force"] * fs.length[fs.fiber][None, :],
                               c["force"] * fs.length[fs.fiber][None, :])


def test_serving_request_ranges():
    for rid in range(20):
        r = W.serving_request(3, rid)
        fs = r["fibers"]
        assert 32 <= fs.n_fib <= 2048
        assert fs.nodes_per_fiber in (16, 32, 64)
        assert 20 <= r["iters"] <= 60
        Rb = 2.0 * fs.n_fib ** (1 / 3)
        centers = fs.xyz.reshape(3, fs.n_fib, fs.nodes_per_fiber).mean(axis=2)
        assert np.linalg.norm(centers, axis=0).max() <= Rb + 1e-9
    t = W.serving_stream(3, 1000, 20.0)
    assert np.all(np.diff(t) > 0) and abs(1000 / t[-1] - 20.0) < 3.0

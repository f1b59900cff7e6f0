"""The seeded input generator: reproducible, normalised, unitary, in range."""
import numpy as np

import qcw_inputs as qi


def test_state_reproducible_and_normalised():
    a = qi.state(1, 10, tag=4)
    b = qi.state(1, 10, tag=4, threads=1)
    assert np.array_equal(a, b)
    assert abs(np.linalg.norm(a) - 1.0) < 1e-14
    assert not np.array_equal(a, qi.state(2, 10, tag=4))


def test_state_chunks_do_not_depend_on_threads():
    # 2^21 amplitudes span two generator chunks
    a = qi.state(3, 21, threads=1)
    b = qi.state(3, 21, threads=4)
    assert np.array_equal(a, b)


def test_random_unitary_is_unitary():
    rng = np.random.default_rng(0)
    for m in (2, 4, 8):
        U = qi.random_unitary(rng, m)
        assert np.max(np.abs(U.conj().T @ U - np.eye(m))) < 1e-14


def test_circuit_draws():
    c = qi.circuit(0, 9, 36)
    assert len(c) == 36
    for k, t, U in zip(c.ks, c.targets, c.mats):
        assert 1 <= k <= 3 and len(set(t)) == k and all(1 <= x <= 9 for x in t)
        assert U.shape == (1 << k, 1 << k)
    c2 = qi.circuit(0, 9, 36)
    assert all(np.array_equal(x, y) for x, y in zip(c.mats, c2.mats))
    small = qi.circuit(0, 1, 10)
    assert set(small.ks) == {1}


def test_batch_sizes_log_uniform():
    nqs = qi.batch_nqs(2, 4096, 3, 7)
    assert nqs.min() == 3 and nqs.max() == 7
    counts = np.bincount(nqs)[3:]
    assert np.all(counts > 700)


def test_poisson_arrivals():
    t = qi.poisson_arrivals(3, 2000.0, 2.0)
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0
    assert 3500 < t.size < 4500


def test_named_gates_unitary():
    for U in (qi.H, qi.X, qi.Y, qi.Z, qi.CNOT, qi.CZ, qi.SWAP, qi.TOFFOLI, qi.cphase(0.3)):
        m = U.shape[0]
        assert np.allclose(U.conj().T @ U, np.eye(m), atol=1e-15)


def test_random_rotation_is_the_exponential_of_a_spin_rotation():
    """UE1-style noise operator: exp(-i theta n.sigma/2) for a unit axis n,
    checked against scipy's matrix exponential of the same generator (theta
    and n read back from the draw order), and SU(2): unitary, det 1."""
    from scipy.linalg import expm
    rng = np.random.default_rng(3)
    for _ in range(20):
        st = rng.bit_generator.state
        R = qi.random_rotation(rng)
        r2 = np.random.default_rng(0)
        r2.bit_generator.state = st
        theta, z, phi = r2.uniform(0, 2 * np.pi), r2.uniform(-1, 1), r2.uniform(0, 2 * np.pi)
        n = np.array([np.sqrt(1 - z * z) * np.cos(phi), np.sqrt(1 - z * z) * np.sin(phi), z])
        G = n[0] * qi.X + n[1] * qi.Y + n[2] * qi.Z
        np.testing.assert_allclose(R, expm(-0.5j * theta * G), rtol=0, atol=1e-14)
        np.testing.assert_allclose(R @ R.conj().T, np.eye(2), rtol=0, atol=1e-14)
        assert abs(np.linalg.det(R) - 1) <= 1e-14


def test_random_rotation_axis_is_isotropic():
    """Axis uniform on the sphere: E[n] = 0 and E[n_i^2] = 1/3, read off the
    rotations themselves (R - R^dagger = -2i sin(theta/2) n.sigma)."""
    rng = np.random.default_rng(4)
    ns = []
    for _ in range(20000):
        R = qi.random_rotation(rng)
        A = (R - R.conj().T) / -2j               # sin(theta/2) n.sigma
        v = np.array([A[0, 1].real, -A[0, 1].imag, A[0, 0].real])
        if np.linalg.norm(v) > 1e-3:
            ns.append(v / np.linalg.norm(v))
    ns = np.array(ns)
    assert np.all(np.abs(ns.mean(axis=0)) < 0.03)
    assert np.all(np.abs((ns ** 2).mean(axis=0) - 1 / 3) < 0.02)

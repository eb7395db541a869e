"""Pins of the oracle's leapfrog (Sect. 3.1) and energy bookkeeping (Eq. (3)),
and of the Plummer generator against the model's closed forms."""

import numpy as np
import pytest

import oracle
import workloads


def _kepler_state():
    # equal masses 1/2 on a circular orbit of separation 1: relative speed 1,
    # period 2 pi sqrt(r^3 / M) = 2 pi
    pos = np.array([[-0.5, 0.0, 0.0], [0.5, 0.0, 0.0]])
    vel = np.array([[0.0, -0.5, 0.0], [0.0, 0.5, 0.0]])
    mass = np.array([0.5, 0.5])
    return pos, vel, mass


def _run(pos, vel, mass, dt, nsteps, theta=0.5, eps=0.0, nleaf=16, ncrit=64):
    pos = pos.copy()
    vel = vel.copy()
    t = oracle.Tree(pos, mass, nleaf, ncrit)
    acc, pot, _, _ = t.forces(theta, eps)
    for _ in range(nsteps):
        oracle.kdk_step(pos, vel, mass, acc, pot, dt, theta, eps, nleaf, ncrit)
    return pos, vel, acc, pot


def test_kepler_period_and_second_order():
    pos0, vel0, m = _kepler_state()
    errs = []
    for nsteps in (400, 800):
        dt = 2 * np.pi / nsteps
        pos, _, _, _ = _run(pos0, vel0, m, dt, nsteps)
        errs.append(np.abs(pos - pos0).max())
    assert errs[0] < 1e-3
    ratio = errs[0] / errs[1]
    assert 3.0 < ratio < 5.0          # error ~ dt^2


def test_time_reversibility():
    pos0, vel0, m = workloads.plummer(48, 9)
    # nleaf >= n: one leaf, all pairs direct, so the force field is smooth
    pos, vel, _, _ = _run(pos0, vel0, m, 1 / 128, 40, eps=0.05, nleaf=64)
    pos, vel, _, _ = _run(pos, -vel, m, 1 / 128, 40, eps=0.05, nleaf=64)
    assert np.abs(pos - pos0).max() < 1e-12
    assert np.abs(vel + vel0).max() < 1e-12


def test_energy_error_is_second_order():
    pos0, vel0, m = workloads.plummer(128, 10)
    eps = 0.05
    t = oracle.Tree(pos0, m, 16, 64)
    _, pot0, _, _ = t.forces(1e-6, eps)
    E0 = oracle.energy(vel0, m, pot0)[2]
    dEs = []
    for dt in (1 / 64, 1 / 128):
        nsteps = int(round(0.5 / dt))
        _, vel, _, pot = _run(pos0, vel0, m, dt, nsteps, theta=1e-6, eps=eps)
        dEs.append(abs((E0 - oracle.energy(vel, m, pot)[2]) / E0))
    assert dEs[0] < 1e-2
    assert 2.5 < dEs[0] / dEs[1] < 6.0


def test_energy_function_parts():
    vel = np.array([[1.0, 2.0, 2.0], [0.0, 0.0, -1.0]])
    mass = np.array([2.0, 4.0])
    pot = np.array([-1.0, -0.5])
    T, W, E, px, py, pz = oracle.energy(vel, mass, pot)
    assert T == 0.5 * 2 * 9 + 0.5 * 4 * 1
    assert W == 0.5 * (2 * -1.0 + 4 * -0.5)
    assert E == T + W
    assert (px, py, pz) == (2.0, 4.0, 0.0)


def test_plummer_sample_matches_model():
    n = 4096
    pos, vel, m = workloads.plummer(n, 1)
    assert m.sum() == pytest.approx(1.0)
    assert np.abs(pos.mean(axis=0)).max() < 1e-14
    assert np.abs(vel.mean(axis=0)).max() < 1e-14
    r = np.sort(np.linalg.norm(pos, axis=1))
    # Henon units: half-mass radius 0.7686 (3 pi / 16 / sqrt(2^(2/3) - 1))
    assert r[n // 2] == pytest.approx(0.7686, rel=0.05)
    _, pot = oracle.direct(pos, m, 0.0)
    T, W, E, _, _, _ = oracle.energy(vel, m, pot)
    assert E == pytest.approx(-0.25, abs=0.02)
    assert 2 * T / abs(W) == pytest.approx(1.0, abs=0.06)

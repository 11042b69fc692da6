"""Pins of the oracle's line search (the energy of the updated state as a
function of the angle, and its minimiser).

* step_energy equals the Rayleigh quotient (Eq. 1) of the fifth-order update
  (Eq. 6) built from dense matrices, renormalised;
* its slope at theta = 0 is the pool gradient of Eq. 5 for that generator;
* line_search's minimiser matches an exhaustive grid on a small register;
* with the exact exponential the energy is a trigonometric polynomial of
  degree two in theta, and the truncated update's energy stays within the
  sixth-order truncation bound of it.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc
from tests.dense_ref import expm_antihermitian, taylor5_dense


def prepared_state(system, steps=2):
    """A state two adaptive steps away from the reference (non-zero gradients)."""
    h = orc.csr_from_pack(system.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in system.pool]
    tr = orc.adapt_run(h, pool, vs.reference_state(system), vs.draw_thetas(system.spec.seed, steps), steps)
    return h, pool, tr.psi


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_step_energy_equals_dense_rayleigh_quotient(mapping):
    s = vs.make_system(vs.SystemSpec(6, 2, mapping, False, 31))
    h, pool, psi = prepared_state(s)
    H = h.dense()
    for k in (0, len(pool) // 2, len(pool) - 1):
        A = pool[k].dense()
        for theta in (-0.7, -0.05, 0.0, 0.13, 0.9):
            phi = taylor5_dense(theta, A) @ psi
            e_dense = np.vdot(phi, H @ phi).real / np.vdot(phi, phi).real
            assert abs(orc.step_energy(h, pool[k], psi, theta) - e_dense) <= 1e-12 * max(1, abs(e_dense))


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_step_energy_slope_is_the_pool_gradient(mapping):
    s = vs.make_system(vs.SystemSpec(8, 4, mapping, False, 32))
    h, pool, psi = prepared_state(s)
    _, _, _, sigma = orc.energy(h, psi)
    g = orc.gradients(pool, psi, sigma)
    eps = 1e-4
    for k in np.argsort(-np.abs(g))[:6]:
        fd = (orc.step_energy(h, pool[k], psi, eps) - orc.step_energy(h, pool[k], psi, -eps)) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_line_search_matches_exhaustive_grid():
    s = vs.make_system(vs.SystemSpec(6, 2, "jw", False, 33))
    h, pool, psi = prepared_state(s, steps=1)
    _, _, _, sigma = orc.energy(h, psi)
    k = int(np.argmax(np.abs(orc.gradients(pool, psi, sigma))))
    theta, e = orc.line_search(h, pool[k], psi, theta_max=1.0)
    grid = np.linspace(-1.0, 1.0, 20001)
    vals = np.array([orc.step_energy(h, pool[k], psi, t) for t in grid])
    i = int(np.argmin(vals))
    assert e <= vals[i] + 1e-13
    assert abs(theta - grid[i]) <= grid[1] - grid[0]
    assert e < orc.step_energy(h, pool[k], psi, 0.0)


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_exact_exponential_energy_is_trigonometric(mapping):
    s = vs.make_system(vs.SystemSpec(6, 2, mapping, True, 34))
    h, pool, psi = prepared_state(s)
    H = h.dense()
    hnorm = np.abs(np.linalg.eigvalsh(H)).max()
    for k in (1, len(pool) - 2):
        A = pool[k].dense()

        def e_exp(t):
            phi = expm_antihermitian(t, A) @ psi
            return np.vdot(phi, H @ phi).real / np.vdot(phi, phi).real

        fit_t = np.array([-1.1, -0.4, 0.2, 0.8, 1.4])
        basis = lambda t: np.stack([np.ones_like(t), np.cos(t), np.sin(t), np.cos(2 * t),
                                    np.sin(2 * t)], axis=-1)
        coef = np.linalg.solve(basis(fit_t), np.array([e_exp(t) for t in fit_t]))
        for t in (-0.9, -0.1, 0.33, 1.2, 2.5):
            assert abs(basis(np.array(t)) @ coef - e_exp(t)) <= 1e-11 * max(1, abs(e_exp(t)))
        # the truncated update: energy error of order theta^6
        for t in (-0.3, -0.1, 0.05, 0.2, 0.4):
            bound = 4 * hnorm * abs(t) ** 6 / 720
            assert abs(orc.step_energy(h, pool[k], psi, t) - e_exp(t)) <= bound + 1e-13


def test_adapt_with_line_search_descends():
    s = vs.make_system(vs.SystemSpec(8, 4, "jw", False, 35))
    h = orc.csr_from_pack(s.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    psi0 = vs.reference_state(s)
    steps = 5
    ls = orc.adapt_run(h, pool, psi0, None, steps, line_search_max=1.0)
    rnd = orc.adapt_run(h, pool, psi0, vs.draw_thetas(s.spec.seed, steps), steps)
    e = np.array(ls.energies)
    assert np.all(np.diff(e) <= 1e-14)
    assert e[-1] < rnd.energies[-1]
    # variational: above the lowest eigenvalue of H
    assert e[-1] >= np.linalg.eigvalsh(h.dense()).min() - 1e-10

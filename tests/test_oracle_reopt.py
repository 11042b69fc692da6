"""Pins of the oracle's re-optimisation of every angle of the adaptive ansatz
(cyclic coordinate minimisation of the ansatz energy).

* ansatz_state is the product of dense fifth-order update matrices (Eq. 6)
  applied to the reference in selection order, up to normalisation;
* one coordinate's new angle matches an exhaustive grid of the dense energy,
  and no visit raises the energy;
* after enough sweeps the angles are a stationary point of the dense energy
  (central differences) and a quasi-Newton minimisation (BFGS) of the dense
  energy over all angles, from the same start, ends at the same energy;
* adaptive runs with re-optimisation reach the exact ground energy of the
  reference's particle sector (dense eigh) on a 6-qubit system, which the
  same number of steps without it does not.
"""
import numpy as np
import pytest

import vqe_system as vs
from oracle import oracle as orc
from tests.dense_ref import taylor5_dense


def setup(n, ne, mapping, seed, steps):
    s = vs.make_system(vs.SystemSpec(n, ne, mapping, False, seed))
    h = orc.csr_from_pack(s.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    ref = vs.reference_state(s)
    tr = orc.adapt_run(h, pool, ref, None, steps, line_search_max=1.0)
    return s, h, pool, ref, tr.selected, np.array(tr.thetas)


def dense_energy(H, D, ref, ks, th):
    phi = np.asarray(ref, dtype=np.complex128)
    for k, t in zip(ks, th):
        phi = taylor5_dense(float(t), D[k]) @ phi
    return np.vdot(phi, H @ phi).real / np.vdot(phi, phi).real


@pytest.mark.parametrize("mapping", ["jw", "bk"])
def test_ansatz_state_is_the_dense_product(mapping):
    s, h, pool, ref, ks, th = setup(6, 2, mapping, 37, 4)
    D = [p.dense() for p in pool]
    th = th + np.array([0.3, -0.2, 0.5, -0.4])        # away from any optimum
    phi = np.asarray(ref, dtype=np.complex128)
    for k, t in zip(ks, th):
        phi = taylor5_dense(float(t), D[k]) @ phi
    psi = orc.ansatz_state(pool, ref, ks, th)
    assert abs(np.vdot(psi, psi).real - 1.0) < 1e-14
    fid = abs(np.vdot(phi, psi)) ** 2 / np.vdot(phi, phi).real
    assert fid > 1 - 1e-14
    e = orc.ansatz_energy(h, pool, ref, ks, th)
    assert abs(e - dense_energy(h.dense(), D, ref, ks, th)) < 1e-12


def test_coordinate_visits_minimise_and_descend():
    s, h, pool, ref, ks, th = setup(6, 2, "jw", 38, 3)
    H, D = h.dense(), [p.dense() for p in pool]
    start = th + np.array([0.25, -0.3, 0.2])
    trace = []
    orc.reoptimize(h, pool, ref, ks, start, sweeps=1, trace=trace)
    e_prev = dense_energy(H, D, ref, ks, start)
    grid = np.linspace(-1.0, 1.0, 4001)
    for m, before, t_new, e_new in trace:
        # the visit's energy is the dense energy at the new angle, no higher
        # than before the visit, and no grid point beats it
        trial = before.copy()
        trial[m] = t_new
        assert abs(dense_energy(H, D, ref, ks, trial) - e_new) < 1e-12
        assert e_new <= e_prev + 1e-14
        vals = []
        for t in grid:
            trial[m] = t
            vals.append(dense_energy(H, D, ref, ks, trial))
        assert e_new <= min(vals) + 1e-13
        e_prev = e_new


@pytest.mark.parametrize("mapping,seed", [("jw", 36), ("bk", 39)])
def test_converged_angles_are_stationary_and_match_bfgs(mapping, seed):
    from scipy.optimize import minimize
    s, h, pool, ref, ks, th0 = setup(6, 2, mapping, seed, 4)
    H, D = h.dense(), [p.dense() for p in pool]
    th = orc.reoptimize(h, pool, ref, ks, th0, sweeps=20)
    f = lambda t: dense_energy(H, D, ref, ks, t)
    eye = np.eye(len(th))
    grad = [(f(th + 1e-5 * eye[i]) - f(th - 1e-5 * eye[i])) / 2e-5 for i in range(len(th))]
    assert np.abs(grad).max() < 1e-6
    res = minimize(f, th0, method="BFGS", options={"gtol": 1e-10})
    assert abs(f(th) - res.fun) < 1e-12
    assert f(th) <= f(th0) + 1e-14


def test_adapt_with_reoptimisation_reaches_the_sector_ground_state():
    n = 6
    s = vs.make_system(vs.SystemSpec(n, 2, "jw", False, 35))
    h = orc.csr_from_pack(s.hamiltonian)
    pool = [orc.csr_from_pack(p) for p in s.pool]
    ref = vs.reference_state(s)
    # the reference's alpha and beta counts fix the sector (spin-orbital 2p +
    # sigma in bit 2p + sigma)
    amask = int("01" * (n // 2), 2)
    bmask = amask << 1
    r = s.reference_index
    na, nb = bin(r & amask).count("1"), bin(r & bmask).count("1")
    idx = [c for c in range(1 << n)
           if bin(c & amask).count("1") == na and bin(c & bmask).count("1") == nb]
    H = h.dense()
    e_exact = np.linalg.eigvalsh(H[np.ix_(idx, idx)]).min()
    steps = 10
    plain = orc.adapt_run(h, pool, ref, None, steps, line_search_max=1.0)
    reopt = orc.adapt_run(h, pool, ref, None, steps, line_search_max=1.0, reopt_sweeps=1)
    assert plain.energies[-1] - e_exact > 1e-5
    assert reopt.energies[-1] - e_exact < 1e-9
    assert reopt.energies[-1] >= e_exact - 1e-12
    # the final state is the ansatz at the final angles
    psi = orc.ansatz_state(pool, ref, reopt.selected, reopt.thetas)
    assert abs(orc.energy(h, psi)[0] - reopt.energies[-1]) < 1e-14

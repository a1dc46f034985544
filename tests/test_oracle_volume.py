"""Pins of the oracle's volumetric ARAP energy (Fig. 31, A.2.5).

* the rest state (offsets at the rest positions, zero angles, targets at rest)
  has E = 0 exactly, and a rigid motion of everything keeps E = 0 to rounding;
* it is the mesh ARAP energy (pinned independently) on the voxel lattice's edge
  list: the two give the same cost, J^T F, diag(J^T J) and J^T J (their residual
  rows come in another order, which these quantities do not see);
* its Jacobian equals central finite differences.
"""
import numpy as np

import oracle
from oracle.energies import ArapVolume, euler_rotate
import workloads as w


def _mesh_twin(d):
    return oracle.ArapMesh(d["W"] * d["H"] * d["D"], w.lattice_edges(d["W"], d["H"], d["D"]), d["U"], d["C"],
                           d["params"]["w_fit"], d["params"]["w_reg"])


def test_rest_state_and_rigid_motion_have_zero_energy():
    d = w.arap_volume(5, 4, 3, seed=1, handle_frac=0.1)
    n = 60
    U = d["U"]
    C = np.where(d["C"] >= -999999.9, U, d["C"])  # targets at rest
    e = ArapVolume(5, 4, 3, U, C, 10.0, 1.0)
    x = np.concatenate([U, np.zeros((3, n))])
    assert oracle.cost(e, x) == 0.0
    a0 = np.array([0.3, -0.2, 0.7])
    R = lambda v: euler_rotate(np.broadcast_to(a0[:, None], v.shape), v)
    t = np.array([[1.5], [-2.0], [0.25]])
    Cm = np.where(d["C"] >= -999999.9, R(U) + t, d["C"])
    e2 = ArapVolume(5, 4, 3, U, Cm, 10.0, 1.0)
    x2 = np.concatenate([R(U) + t, np.repeat(a0[:, None], n, 1)])
    assert oracle.cost(e2, x2) < 1e-24


def test_equals_mesh_energy_on_the_lattice():
    d = w.arap_volume(6, 5, 4, seed=2, handle_frac=0.05)
    ev, em = oracle.make_energy(d), _mesh_twin(d)
    rng = np.random.default_rng(5)
    x = d["x0"].ravel() + 0.1 * rng.normal(size=d["x0"].size)
    lv, lm = oracle.Linearization(ev, x), oracle.Linearization(em, x)
    assert abs(lv.E - lm.E) <= 1e-13 * lm.E
    assert np.allclose(lv.jtf(), lm.jtf(), rtol=0, atol=1e-12 * np.abs(lm.jtf()).max())
    assert np.allclose(lv.diag, lm.diag, rtol=0, atol=1e-12 * lm.diag.max())
    A1 = (lv.JT @ lv.J).toarray()
    A2 = (lm.JT @ lm.J).toarray()
    assert np.allclose(A1, A2, rtol=0, atol=1e-12 * np.abs(A2).max())


def test_jacobian_matches_finite_differences():
    d = w.arap_volume(3, 3, 2, seed=3, handle_frac=0.2)
    e = oracle.make_energy(d)
    x = d["x0"].ravel() + 0.2 * np.random.default_rng(1).normal(size=d["x0"].size)
    J = oracle.jacobian(e, x).toarray()
    Jfd = oracle.fd_jacobian(e, x)
    assert np.abs(J - Jfd).max() <= 1e-6 * max(1.0, np.abs(J).max())


def test_workload_anchors_the_bottom_face():
    d = w.arap_volume(4, 3, 5, seed=4, handle_frac=0.0)
    base = np.arange(12)
    assert np.array_equal(d["C"][:, base], d["U"][:, base])
    assert len(d["handles"]) == 1  # at least one handle besides the anchored face

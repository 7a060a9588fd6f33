"""Host-side metrics: the scale-free symplectic defect of the monodromy."""
import numpy as np

from paper_2601_17164_amd import metrics


def _states(Ms):
    """Final-state layout y[43][n] with the monodromy columns (Q(3), P(3)) at rows 6..41."""
    n = len(Ms)
    y = np.zeros((43, n))
    for j, M in enumerate(Ms):
        y[6:42, j] = M.T.reshape(-1)  # column c of M at rows 6 + 6c .. 6 + 6c + 5
    return y


def test_symplectic_defect():
    rng = np.random.default_rng(1)
    A = rng.normal(size=(3, 3)) + 3 * np.eye(3)
    S = rng.normal(size=(3, 3))
    S = S + S.T
    lift = np.block([[A, np.zeros((3, 3))], [np.zeros((3, 3)), np.linalg.inv(A).T]])
    shear = np.block([[np.eye(3), 1e3 * S], [np.zeros((3, 3)), np.eye(3)]])
    good = [np.eye(6), lift, shear @ lift]          # symplectic, the last with ||M|| ~ 1e4
    bad = lift.copy()
    bad[0, 0] *= 1.0 + 1e-4  # no longer symplectic (||M|| ~ 5: the defect shows at its scale)
    d = metrics.symplectic_defect(_states(good + [bad]))
    assert d[0] == 0.0 and np.all(d[1:3] < 1e-15)
    assert d[3] > 1e-6

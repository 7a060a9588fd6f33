"""Fit the synthetic ground-state GTO expansions used by the synthetic workloads.

The paper expands psi_0 in Gaussian-type orbitals whose exponents are kept fixed and whose
coefficients are fitted by linear regression to the time-independent ground state (App. B.1).
Its fitted coefficients are not printed, so this script makes stand-in fits of the same kind:

* ``gto_s_h1s.json``: s-wave, sum_j c_j exp(-a_j r^2) fitted to the hydrogen 1s state
  pi^{-1/2} exp(-r), least squares with weight r^2 dr on r in [0, 20];
* ``gto_p_ip058.json``: p-wave, z sum_j c_j exp(-a_j r^2) fitted to the normalised
  z exp(-kappa r), kappa = sqrt(2 * 0.58), weight r^4 dr on r in [0, 20].

Both use the six even-tempered exponents a_j = 0.03 * 3.5^j, j = 0..5. Run once; the JSON files
are inputs read by both the oracle-side tests and the HIP path.
"""
import json
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ALPHA = [0.03 * 3.5 ** j for j in range(6)]


def _fit(target, radial_weight_power):
    r = np.linspace(0.0, 20.0, 20001)
    w = np.sqrt(r ** radial_weight_power)
    A = np.exp(-np.outer(r * r, ALPHA)) * w[:, None]
    b = target(r) * w
    c, *_ = np.linalg.lstsq(A, b, rcond=None)
    fit = np.exp(-np.outer(r * r, ALPHA)) @ c
    rel = np.linalg.norm((fit - target(r)) * w) / np.linalg.norm(target(r) * w)
    cond = np.linalg.cond(A)
    return c, rel, cond


def main():
    cs, rel_s, cond_s = _fit(lambda r: np.exp(-r) / math.sqrt(math.pi), 2)
    kappa = math.sqrt(2.0 * 0.58)
    # norm of z exp(-kappa r): (4 pi / 3) * 24 / (2 kappa)^5
    nrm = math.sqrt((4.0 * math.pi / 3.0) * 24.0 / (2.0 * kappa) ** 5)
    cp, rel_p, cond_p = _fit(lambda r: np.exp(-kappa * r) / nrm, 4)
    out = {
        "gto_s_h1s.json": {"l": 0, "ip": 0.5, "alpha": ALPHA, "coef": cs.tolist(),
                           "target": "pi^-1/2 exp(-r)", "fit_rel_l2": rel_s, "cond": cond_s},
        "gto_p_ip058.json": {"l": 1, "ip": 0.58, "alpha": ALPHA, "coef": cp.tolist(),
                             "target": "z exp(-kappa r)/norm, kappa=sqrt(2*0.58)",
                             "fit_rel_l2": rel_p, "cond": cond_p},
    }
    for name, data in out.items():
        with open(os.path.join(HERE, name), "w") as f:
            json.dump(data, f, indent=1)
        print(name, "rel L2", data["fit_rel_l2"], "cond", data["cond"])


if __name__ == "__main__":
    main()

"""Write closed_forms.json: traces of inverses of shifted Dirichlet Laplacians.

The unscaled d-dimensional Dirichlet Laplacian on an m^d grid (diagonal 2d,
off-diagonal -1) is a Kronecker sum of tridiag(-1, 2, -1) of order m, whose
eigenvalues are 4 sin^2(j pi / (2 (m + 1))), j = 1..m.  Hence

    tr (A + sigma I)^{-1} = sum_{j in [1, m]^d} 1 / (sum_k 4 sin^2(j_k pi / (2 (m + 1))) + sigma).

Used for the C1 workload (2-D, m = 31, sigma = 0.1: the 5-point stencil with
diagonal 4.1) and for small 3-D unit-weight instances of the C2 family.
Computed with mpmath at 40 digits; needs nothing from the library or oracle.
"""

import itertools
import json
import os

import mpmath as mp

mp.mp.dps = 40


def trace(m, d, sigma):
    lam = [4 * mp.sin(j * mp.pi / (2 * (m + 1))) ** 2 for j in range(1, m + 1)]
    tot = mp.mpf(0)
    for js in itertools.product(range(m), repeat=d):
        tot += 1 / (sum(lam[j] for j in js) + sigma)
    return tot


def main():
    cases = {
        "C1_2d_m31_sigma0.1": (31, 2, mp.mpf("0.1")),
        "3d_m10_sigma0.05": (10, 3, mp.mpf("0.05")),
        "3d_m14_sigma0.05": (14, 3, mp.mpf("0.05")),
    }
    out = {k: {"m": m, "d": d, "sigma": float(s), "trace": mp.nstr(trace(m, d, s), 30)}
           for k, (m, d, s) in cases.items()}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path)


if __name__ == "__main__":
    main()

"""Cost of even-odd preconditioning for the staggered Wilson matrix (oracle study).

Test infrastructure only; run as ``python -m oracle.study_sw_evenodd`` from the
repository root.  On an 8^4 near-identity SU(3) field of the plaquette used for
the benchmark workload (0.594), with m_c found by the oracle's search and a
point source, it prints for m = m_c + delta:

* the eigenvalues of the odd-site diagonal block A_oo = (m + r) - r Gamma_55
  nearest zero and largest in modulus (it is hermitian and indefinite);
* CG iterations of eq. (2) without preconditioning;
* CG iterations on the Schur complement's normal equations S^2 x_e = S b^_e with
  every A_oo^{-1} an inner CG on A_oo^2 to 1e-10, the inner A_oo applications,
  and eq. (2)'s residual of the reconstructed x;
* both costs in Gamma_55 sweeps over one parity (the dominant part of a
  staggered Wilson matvec), and their ratio.
"""
from __future__ import annotations

import sys
import time

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import eigsh

import synth

from . import critical, evenodd_sw, staggered_wilson

DIMS = (8, 8, 8, 8)
EPS = 0.4359375
DELTAS = (0.1, 0.05, 0.02)
TOL = 1e-8
INNER_TOL = 1e-10


def main(deltas=DELTAS):
    U = synth.gauge_field(DIMS, "near_identity", 2000, EPS)
    W = staggered_wilson.corners(U)
    v0 = synth.gaussian_field(DIMS, synth.STAGGERED_WILSON, 7)
    t = time.time()
    mc, _, _ = critical.critical_mass(synth.STAGGERED_WILSON, U, v0, -0.7, -0.3, corners=W)
    print(f"8^4 near-identity field, m_c = {mc:.6f} ({time.time() - t:.0f} s)", flush=True)
    # M depends on m only through m times the identity.
    M0 = evenodd_sw.Blocks(U, 0.0).M
    ident = sp.identity(M0.shape[0], dtype=np.complex128, format="csr")
    chi = synth.point_source(DIMS, synth.STAGGERED_WILSON, 0).ravel()
    rows = []
    for d in deltas:
        m = mc + d
        B = evenodd_sw.Blocks(U, m, M=(M0 + m * ident).tocsr())
        lo = np.abs(eigsh(B.Aoo, k=1, sigma=0.0, which="LM", return_eigenvectors=False)).min()
        hi = np.abs(eigsh(B.Aoo, k=1, which="LM", return_eigenvectors=False)).max()
        _, it, res_u = evenodd_sw.unpreconditioned(B, chi, TOL)
        t = time.time()
        _, info = evenodd_sw.solve(B, chi, TOL, INNER_TOL)
        g, _ = evenodd_sw.cost_in_half_sweeps(info["outer_applications"],
                                              info["inner_applications"])
        gu, _ = evenodd_sw.unpreconditioned_cost(it)
        row = dict(delta=d, m=m, aoo_min=lo, aoo_max=hi, kappa_aoo=hi / lo, unprec_iterations=it,
                   unprec_eq2_residual=res_u, outer_iterations=info["outer_iterations"],
                   inner_per_solve=info["inner_applications"] / info["inner_solves"],
                   eq2_residual=info["eq2_residual"], g55_sweeps=g, g55_sweeps_unprec=gu,
                   cost_ratio=g / gu)
        rows.append(row)
        print(" ".join(f"{k}={v:.4g}" if isinstance(v, float) else f"{k}={v}"
                       for k, v in row.items()), f"({time.time() - t:.0f} s)", flush=True)
    return rows


if __name__ == "__main__":
    main(tuple(float(a) for a in sys.argv[1:]) or DELTAS)

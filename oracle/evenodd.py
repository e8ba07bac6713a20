"""Even-odd (Schur complement) preconditioned CG for the Wilson matrix (oracle).

Test infrastructure only: the library's solvers never call this module.

The paper solves eq. (2) without preconditioning and remarks, in the footnote
to eq. (2) (Sec. 3), that preconditioning would make the Wilson inversion more
than twice as fast.  It does not say which preconditioning; the reading taken
here is the usual even-odd one.  With sites split by the parity of
x1 + x2 + x3 + x4, the hops of M_W = (m + 4r) - (1/2) H only connect opposite
parities, so in (even, odd) blocks

    M_W = [[d, M_eo], [M_oe, d]],   d = m + 4r  (times the identity),

and eliminating the odd half leaves the Schur complement on the even sites,

    M^ = d - M_eo M_oe / d,    M^ x_e = b^_e = chi_e - M_eo chi_o / d,
    x_o = (chi_o - M_oe x_e) / d.

M^ x_e = b^_e is solved by CG on its normal equations M^dag M^ x_e = M^dag b^_e,
the same method as eq. (2) on half the sites.  M^dag = d - M_oe^dag M_eo^dag / d
is M^ built from M_W^dag.  Fields are full-lattice arrays whose odd half is zero
(the even half alone carries x_e); every block is taken from the full operator
by projecting onto a parity, so nothing here restates the hop.
"""
from __future__ import annotations

import numpy as np

from . import lattice, solvers, wilson

import synth

EVEN, ODD = 0, 1


def parity(dims):
    """(x1 + x2 + x3 + x4) mod 2 of every site, site-shaped."""
    x1, x2, x3, x4 = lattice.coords(dims)
    return (x1 + x2 + x3 + x4) & 1


def project(psi, par):
    """psi on the sites of parity `par`, zero elsewhere."""
    mask = parity(lattice.dims_of(psi)) == par
    return psi * mask.reshape(mask.shape + (1,) * (psi.ndim - 4))


def schur_apply(U, xe, m, bc=(1, 1, 1, 1), dagger=False):
    """M^ x_e (or M^dag x_e) for x_e zero on the odd sites; r = 1."""
    d = m + 4.0
    moe = project(wilson.apply(U, xe, m, 1.0, bc, dagger), ODD)     # M_oe x_e
    meo = project(wilson.apply(U, moe, m, 1.0, bc, dagger), EVEN)   # M_eo M_oe x_e
    return d * xe - meo / d


def rhs(U, chi, m, bc=(1, 1, 1, 1)):
    """b^_e = chi_e - M_eo chi_o / d."""
    d = m + 4.0
    chi_o = project(chi, ODD)
    return project(chi, EVEN) - project(wilson.apply(U, chi_o, m, 1.0, bc), EVEN) / d


def reconstruct(U, xe, chi, m, bc=(1, 1, 1, 1)):
    """The full solution x = x_e + x_o, x_o = (chi_o - M_oe x_e) / d."""
    d = m + 4.0
    xo = (project(chi, ODD) - project(wilson.apply(U, xe, m, 1.0, bc), ODD)) / d
    return project(xe, EVEN) + xo


def cgnr(U, chi, m, tol, maxiter, bc=(1, 1, 1, 1)):
    """Even-odd preconditioned solve of M_W x = chi.

    CG on M^dag M^ x_e = M^dag b^_e to ||r|| / ||M^dag b^_e|| <= tol (the
    stopping rule of ``solvers.cg``), then the odd half by reconstruction.
    info gains ``full_residual``: ||b - A x|| / ||b|| of eq. (2) for the full x.
    """
    Mh = lambda v: schur_apply(U, v, m, bc)
    Mhd = lambda v: schur_apply(U, v, m, bc, dagger=True)
    b = Mhd(rhs(U, chi, m, bc))
    xe, info = solvers.cg(lambda v: Mhd(Mh(v)), b, tol, maxiter)
    x = reconstruct(U, xe, chi, m, bc)
    info["b_norm"] = np.sqrt(float(np.vdot(b.ravel(), b.ravel()).real))
    info["full_residual"] = solvers.true_residual(synth.WILSON, U, chi, x, m, 1.0, bc)[0]
    return x, info

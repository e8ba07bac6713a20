"""Even-odd block elimination for the staggered Wilson matrix (oracle, study).

Test infrastructure only: the library's solvers never call this module.

The footnote to eq. (2) (Sec. 3) expects preconditioning to speed up the Wilson
inversion by more than a factor 2; the paper does not apply it to staggered
Wilson fermions.  This module takes the even-odd Schur complement of M_SW as far
as it goes, to measure what it would cost.

Parity structure.  With sites split by the parity of x1 + x2 + x3 + x4, the
staggered hops of D_st connect opposite parities, but Gamma_55 -- a product of
one shift in each of the four directions -- moves every coordinate by one, so
it keeps the parity.  In (even, odd) blocks

    M_SW = [[A_ee, D_eo], [D_oe, A_oo]],   A = (m + r) - r Gamma_55,

and the diagonal blocks are not multiples of the identity.  Gamma_55 is
hermitian and D_st anti-hermitian (D_oe = -D_eo^dag), so the Schur complement
on the even sites,

    S = A_ee - D_eo A_oo^{-1} D_oe = A_ee + D_eo A_oo^{-1} D_eo^dag,
    S x_e = chi_e - D_eo A_oo^{-1} chi_o,   x_o = A_oo^{-1} (chi_o - D_oe x_e),

is hermitian, and every application of S needs one solve with A_oo.  A_oo is
hermitian with the eigenvalues m + r - r g, g over the spectrum of Gamma_55 on
the odd sites, which lies in [-1, 1] (at U = 1 it is +-prod_mu cos p_mu, the
closed form of ``spectrum.sw_free_real_imag``).  Near the critical mass
m + r is about r/2, inside that range, so A_oo is indefinite and has
eigenvalues near zero: the inner solve is itself ill-conditioned.

Here everything acts on flattened canonical fields through a sparse matrix of
M_SW recovered from the oracle's own matvec by probing (``sparse_matrix``), so
the blocks are index slices and no part of the operator is written again.
The outer solve is CG on S^dag S = S^2 (the normal equations, as in eq. (2));
the inner solves are CG on A_oo^2 (its normal equations).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

from . import lattice, solvers, staggered_wilson

# The displacements of M_SW: the site itself, the 8 hops of D_st and the 16
# corners x + s, s in {+-1}^4, of Gamma_55 (Sec. 3: 8 + 16 other sites).
DISPLACEMENTS = ([(0, 0, 0, 0)]
                 + [tuple(sg if nu == mu else 0 for nu in range(4))
                    for mu in range(4) for sg in (1, -1)]
                 + list(itertools.product((1, -1), repeat=4)))


def _probe_period(L):
    """Smallest k >= 3 dividing L: sites whose coordinates agree mod k then never
    both lie within distance 1 of one site, so one probe per residue class
    recovers every column."""
    for k in range(3, L + 1):
        if L % k == 0:
            return k
    return L


def sparse_matrix(op, dims, inner=3):
    """CSR matrix of ``op`` (a linear map on canonical fields of shape
    site_shape + (inner,)) whose range at x involves only x + DISPLACEMENTS.

    Probe c has ones on component a of every site whose coordinates are
    congruent to c modulo the probe periods; row x of op(probe) then holds the
    column of the one site x + s of that class."""
    x = lattice.coords(dims)
    ks = [_probe_period(L) for L in dims]
    V = int(np.prod(dims))
    site = np.arange(V).reshape(x[0].shape)
    rows, cols, vals = [], [], []
    classes = list(itertools.product(*[range(k) for k in ks]))
    for c in classes:
        member = np.ones(x[0].shape, dtype=bool)
        for mu in range(4):
            member &= (x[mu] % ks[mu]) == c[mu]
        for a in range(inner):
            probe = np.zeros(x[0].shape + (inner,), dtype=np.complex128)
            probe[member, a] = 1.0
            R = op(probe).reshape(V, inner)
            for s in DISPLACEMENTS:
                y = [(x[mu] + s[mu]) % dims[mu] for mu in range(4)]
                hit = np.ones(x[0].shape, dtype=bool)
                for mu in range(4):
                    hit &= (y[mu] % ks[mu]) == c[mu]
                if not hit.any():
                    continue
                src = site.ravel()[hit.ravel()]
                dst = site[y[3], y[2], y[1], y[0]].ravel()[hit.ravel()]
                for b in range(inner):
                    rows.append(src * inner + b)
                    cols.append(dst * inner + a)
                    vals.append(R[src, b])
    n = V * inner
    M = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    M.sum_duplicates()
    return M


def parity_index(dims, inner=3):
    """Flattened component indices of the even and of the odd sites."""
    x1, x2, x3, x4 = lattice.coords(dims)
    par = ((x1 + x2 + x3 + x4) & 1).ravel()
    comp = np.arange(par.size * inner).reshape(par.size, inner)
    return comp[par == 0].ravel(), comp[par == 1].ravel()


class Blocks:
    """The four parity blocks of M_SW at mass m (sparse, CSR)."""

    def __init__(self, U, m, r=1.0, bc=(1, 1, 1, 1), M=None):
        dims = lattice.dims_of(U)
        if M is None:
            W = staggered_wilson.corners(U)
            M = sparse_matrix(lambda v: staggered_wilson.apply(
                U, v, m, r, bc, g55=staggered_wilson.gamma55_corners(W, v, bc)), dims)
        self.dims, self.m, self.r, self.M = dims, m, r, M
        self.e, self.o = parity_index(dims)
        self.Aee = M[self.e][:, self.e].tocsr()
        self.Aoo = M[self.o][:, self.o].tocsr()
        self.Deo = M[self.e][:, self.o].tocsr()
        self.Doe = M[self.o][:, self.e].tocsr()


def inner_solve(B, z, tol, maxiter=100000):
    """y = A_oo^{-1} z and the number of A_oo applications it took: CG on
    A_oo^2 y = A_oo z (A_oo hermitian, so A_oo^dag A_oo = A_oo^2), stopped by the
    oracle CG's rule at ||r|| <= tol ||A_oo z||; two applications per iteration
    plus the right-hand side."""
    A = B.Aoo
    b = A @ z
    y, info = solvers.cg(lambda v: A @ (A @ v), b, tol, maxiter)
    return y, 2 * info["applications"] + 1


class Schur:
    """S v = A_ee v - D_eo A_oo^{-1} D_oe v with counted inner solves."""

    def __init__(self, B, inner_tol):
        self.B, self.tol = B, inner_tol
        self.inner_apps = 0
        self.inner_solves = 0

    def ainv(self, z):
        y, n = inner_solve(self.B, z, self.tol)
        self.inner_apps += n
        self.inner_solves += 1
        return y

    def __call__(self, v):
        B = self.B
        return B.Aee @ v - B.Deo @ self.ainv(B.Doe @ v)


def solve(B, chi, tol, inner_tol, maxiter=100000):
    """Even-odd solve of M_SW x = chi (chi flattened) through the Schur complement.

    CG on S^2 x_e = S b^_e (S hermitian) to the oracle CG's stopping rule,
    then x_o.  Returns x and a dict with the outer iterations, the inner
    solves and A_oo applications, and eq. (2)'s relative residual
    ||M^dag (chi - M x)|| / ||M^dag chi|| of the full x."""
    S = Schur(B, inner_tol)
    bhat = chi[B.e] - B.Deo @ S.ainv(chi[B.o])
    rhs = S(bhat)
    xe, info = solvers.cg(lambda v: S(S(v)), rhs, tol, maxiter)
    xo = S.ainv(chi[B.o] - B.Doe @ xe)
    x = np.zeros_like(chi)
    x[B.e] = xe
    x[B.o] = xo
    Mh = B.M.conj().T
    res = np.linalg.norm(Mh @ (chi - B.M @ x)) / np.linalg.norm(Mh @ chi)
    return x, dict(outer_iterations=info["iterations"], outer_applications=info["applications"],
                   inner_solves=S.inner_solves, inner_applications=S.inner_apps,
                   eq2_residual=float(res), status=info["status"])


def unpreconditioned(B, chi, tol, maxiter=100000):
    """CG on eq. (2) with the same sparse matrix: (x, iterations, eq. (2) residual)."""
    Mh = B.M.conj().T
    b = Mh @ chi
    x, info = solvers.cg(lambda v: Mh @ (B.M @ v), b, tol, maxiter)
    res = np.linalg.norm(b - Mh @ (B.M @ x)) / np.linalg.norm(b)
    return x, info["iterations"], float(res)


def cost_in_half_sweeps(outer_apps, inner_apps):
    """(Gamma_55, D_st) applications over one parity for the even-odd solve.

    Each S application is one A_ee (one Gamma_55 sweep of the even sites), D_oe
    and D_eo (one D_st sweep each) and one inner solve; every A_oo application
    is one Gamma_55 sweep of the odd sites.  The right-hand side and x_o add
    two inner solves (counted in inner_apps) and two D_st sweeps."""
    s_apps = 2 * outer_apps + 1   # S^2 per CG application, plus S b^_e
    return s_apps + inner_apps, 2 * s_apps + 2


def unpreconditioned_cost(iterations):
    """(Gamma_55, D_st) half-lattice sweeps of unpreconditioned CG: M and M^dag
    per iteration, each one full-lattice sweep of both (two half sweeps)."""
    return 4 * (iterations + 1), 4 * (iterations + 1)

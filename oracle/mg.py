"""Oracle: Kahler-Dirac adaptive multigrid (setup and K-cycle solve), FP64.

TEST INFRASTRUCTURE ONLY (see oracle/staggered.py).

Follows Sec. 3 (Galerkin coarsening with chirally doubled, block-orthonormal
near-null vectors, R = P^dag) and Sec. 4 with the parameters of Table 1:

setup (Sec. 4, itemised steps; Table 1 "setup" rows), per coarsening level:
  1. for each of n_vec Gaussian starts psi0: CG on A A^dag e = -A A^dag psi0
     to relative residual 1e-4 or 250 iterations; psi = psi0 + e;
  2. orthonormalise the n_vec vectors globally (modified Gram-Schmidt in
     vector order);
  3. chirally double with (1 +- epsilon)/2 (level 1) or (1 +- sigma_3)/2
     (coarser levels) and orthonormalise within every (aggregate, chirality)
     by a thin QR with positive real diagonal -> P, with P^dag P = 1;
  4. coarse operator A_hat = P^dag A P.

solve (Sec. 4 and Table 1 "solver" rows):
  * level 1: flexible GCR(32) on the KD-block-parity Schur operator
    S = 1 - A_eo A_oe, stopping at ||b - D x|| <= tol ||b||;
  * preconditioner: K-cycle = MR(2, omega 0.85) pre-smooth, restrict,
    approximate coarse solve, prolong, MR(2, 0.85) post-smooth.  On level 1
    the restriction treats the odd-block residual as zero and only the
    even-block part of the prolonged correction is used;
  * intermediate levels: GCR(8) on A_hat, at most 16 iterations, tolerance 0.2,
    itself preconditioned by the next K-cycle;
  * coarsest level: CGNE (CG on A A^dag, x = A^dag y), tolerance 0.2, at most 256.
    Option beyond the paper (``MGParams.coarse_exact``): the coarsest system
    is solved exactly, by a dense LU factorisation of the coarsest operator
    made once per hierarchy, instead of CGNE(0.2).

Null vectors are random by construction, so their values are parity unpinned
against the paper; everything downstream of them (P, A_hat, the solve) is
pinned given them.
"""
from dataclasses import dataclass, field
import numpy as np
import scipy.linalg
import scipy.sparse as sp

from .kd import KDOperator
from .staggered import epsilon


# ---------------------------------------------------------------- parameters

@dataclass
class LevelParams:
    agg: tuple            # aggregate extent per direction (KD blocks on level 1)
    nvec: int             # near-null vectors generated on this level


@dataclass
class MGParams:
    levels: list = field(default_factory=lambda: [LevelParams((4, 4), 8),
                                                  LevelParams((2, 2), 12)])
    setup_tol: float = 1e-4
    setup_maxit: int = 250
    outer_restart: int = 32
    outer_maxit: int = 2000
    mr_its: int = 2
    mr_omega: float = 0.85
    inter_restart: int = 8
    inter_maxit: int = 16
    inter_tol: float = 0.2
    coarse_tol: float = 0.2
    coarse_maxit: int = 256
    coarse_exact: bool = False   # dense LU solve on the coarsest level (not the paper's CGNE)
    fine_schur: bool = True      # level 1 on the KD-block-parity Schur system (False: on the full A)
    fine_op: str = "A"           # operator coarsened and solved: "A" = D B^-1 (the paper's method);
                                 # "D" = the staggered D itself, the naive Galerkin MG of Sec. 3.2
    asymmetric: bool = False     # R != P^dag: chiral doubling with gamma_5^{L/R} and block
                                 # bi-orthonormalisation on every coarsening (Sec. 5, App. A)


def vdot(a, b):
    return np.vdot(a, b)


def norm(a):
    return float(np.sqrt(np.vdot(a, a).real))


# ---------------------------------------------------------------- setup

def cg(apply, b, tol, maxit):
    """Conjugate gradient for Hermitian positive definite ``apply``; x0 = 0.

    Stops when ||r|| <= tol ||b|| or after ``maxit`` iterations.
    """
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = vdot(r, r).real
    bnorm = np.sqrt(rr)
    its = 0
    if bnorm == 0.0:
        return x, 0
    while its < maxit:
        q = apply(p)
        alpha = rr / vdot(p, q).real
        x += alpha * p
        r -= alpha * q
        its += 1
        rr_new = vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bnorm:
            break
        p = r + (rr_new / rr) * p
        rr = rr_new
    return x, its


def relax_null_vectors(op, psi0, tol, maxit):
    """Sec. 4: psi = psi0 + e with A A^dag e = -A A^dag psi0 relaxed by CG."""
    opH = op.conj().T.tocsr()
    normal = lambda v: op @ (opH @ v)
    out = []
    its = []
    for v0 in psi0:
        r = -normal(v0)
        e, k = cg(normal, r, tol, maxit)
        out.append(v0 + e)
        its.append(k)
    return np.array(out), its


def global_orthonormalise(vecs):
    """Modified Gram-Schmidt over the whole lattice, in vector order."""
    V = np.array(vecs, dtype=np.complex128)
    for i in range(V.shape[0]):
        for j in range(i):
            V[i] -= vdot(V[j], V[i]) * V[j]
        V[i] /= norm(V[i])
    return V


def thin_qr_positive(M):
    """Thin QR with a positive real diagonal of R (unique for full rank M)."""
    Q, R = np.linalg.qr(M)
    d = np.diagonal(R)
    ph = d / np.abs(d)
    return Q * ph[None, :]


@dataclass
class Aggregation:
    agg_of_dof: np.ndarray     # aggregate (coarse site) of every fine dof
    chir_of_dof: np.ndarray    # 0 for chirality +1, 1 for -1
    coarse_dims: tuple
    n_coarse_sites: int


def aggregation_level1(lat, agg):
    """Aggregates of agg_mu KD blocks (2*agg_mu sites) per direction; chirality
    from epsilon(x)."""
    size = 2 * np.array(agg)
    cdims = tuple(int(L // s) for L, s in zip(lat.dims, size))
    zc = lat.coords // size
    strides = np.cumprod((1,) + cdims[:-1])
    z = (zc * strides).sum(axis=1)
    chir = np.where(epsilon(lat) > 0, 0, 1)
    nc = lat.ncolor
    return Aggregation(np.repeat(z, nc), np.repeat(chir, nc), cdims,
                       int(np.prod(cdims)))


def aggregation_coarse(dims, ndof_site, nvec_prev, agg):
    """Aggregates of agg_mu coarse sites; chirality from sigma_3, i.e. the
    first nvec_prev dofs of a site are +1, the rest -1."""
    dims = tuple(dims)
    nsite = int(np.prod(dims))
    coords = np.empty((nsite, len(dims)), dtype=np.int64)
    rem = np.arange(nsite)
    for mu, L in enumerate(dims):
        coords[:, mu] = rem % L
        rem //= L
    a = np.array(agg)
    cdims = tuple(int(L // s) for L, s in zip(dims, a))
    strides = np.cumprod((1,) + cdims[:-1])
    z = ((coords // a) * strides).sum(axis=1)
    d = np.arange(ndof_site)
    chir = np.where(d < nvec_prev, 0, 1)
    return Aggregation(np.repeat(z, ndof_site), np.tile(chir, nsite), cdims,
                       int(np.prod(cdims)))


def prolongator(vecs, aggr):
    """Chirally doubled, block-orthonormalised prolongator (sparse n_f x n_c).

    Column index of (aggregate Z, chirality c, vector i) is Z*2n + c*n + i.
    """
    nvec = vecs.shape[0]
    nf = vecs.shape[1]
    rows, cols, vals = [], [], []
    key = aggr.agg_of_dof * 2 + aggr.chir_of_dof
    order = np.argsort(key, kind="stable")
    bounds = np.searchsorted(key[order], np.arange(2 * aggr.n_coarse_sites + 1))
    for zc in range(2 * aggr.n_coarse_sites):
        dofs = order[bounds[zc]:bounds[zc + 1]]
        if dofs.size < nvec:
            raise ValueError("aggregate-chirality smaller than n_vec")
        Q = thin_qr_positive(vecs[:, dofs].T)
        z, c = divmod(zc, 2)
        for i in range(nvec):
            rows.append(dofs)
            cols.append(np.full(dofs.size, z * 2 * nvec + c * nvec + i))
            vals.append(Q[:, i])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                                  np.concatenate(cols))),
                         shape=(nf, aggr.n_coarse_sites * 2 * nvec)).tocsr()


def galerkin(P, A, R=None):
    """A_hat = R A P with R = P^dag unless given."""
    R = P.conj().T if R is None else R
    return (R @ (A @ P)).tocsr()


def lu_nopivot(M):
    """M = L U with L unit lower and U upper triangular, no pivoting
    (Doolittle), as the thin-LU of Sec. 5 (eq. thinlu)."""
    n = M.shape[0]
    L = np.eye(n, dtype=np.complex128)
    U = np.array(M, dtype=np.complex128)
    for k in range(n):
        if U[k, k] == 0:
            raise np.linalg.LinAlgError("zero pivot in the thin LU")
        for i in range(k + 1, n):
            L[i, k] = U[i, k] / U[k, k]
            U[i, k:] -= L[i, k] * U[k, k:]
    return L, np.triu(U)


def asymmetric_transfer(V, Vbar, aggr, gL, gR):
    """Asymmetric coarsening (Sec. 5, eqs. prcplx and thinlu; App. A).

    V, Vbar: right and left vectors [nvec][n_f]; gL, gR: the operator pair of
    the level (gamma_5^L = eps B^-1 and gamma_5^R = B eps on the fine level,
    sigma_1^{L/R} on coarser ones), local to aggregates.  Per aggregate Z:
      R~ = [ Vbar_i^dag ; V_i^dag gL ] (rows),  P~ = [ V_i , gR Vbar_i ] (columns),
      R~ P~ = L U (thin LU),  R = L^-1 R~,  P = P~ U^-1  (so R P = 1),
    and the coarse pair sigma_1^L = U^-dag sigma_1 L, sigma_1^R = U sigma_1 L^-dag,
    with sigma_1 exchanging the two halves.  Coarse dof order per aggregate:
    the n_vec V-columns, then the n_vec gR Vbar columns.
    Returns sparse P (n_f x n_c), R (n_c x n_f), sigma_1^L, sigma_1^R."""
    nvec, nf = V.shape
    nz = aggr.n_coarse_sites
    nd = 2 * nvec
    gRVb = (gR @ Vbar.T).T            # [nvec][n_f]: gR Vbar_i
    VgL = (gL.T @ V.conj().T).T       # [nvec][n_f]: the rows V_i^dag gL
    s1 = np.block([[np.zeros((nvec, nvec)), np.eye(nvec)], [np.eye(nvec), np.zeros((nvec, nvec))]])
    order = np.argsort(aggr.agg_of_dof, kind="stable")
    bounds = np.searchsorted(aggr.agg_of_dof[order], np.arange(nz + 1))
    pr, pc, pv, rr, rc, rv = [], [], [], [], [], []
    sl = np.zeros((nz, nd, nd), dtype=np.complex128)
    sr = np.zeros((nz, nd, nd), dtype=np.complex128)
    for z in range(nz):
        dofs = order[bounds[z]:bounds[z + 1]]
        Rt = np.vstack([Vbar[:, dofs].conj(), VgL[:, dofs]])       # nd x |Z|
        Pt = np.hstack([V[:, dofs].T, gRVb[:, dofs].T])            # |Z| x nd
        L, Uu = lu_nopivot(Rt @ Pt)
        Rz = np.linalg.solve(L, Rt)
        Pz = Pt @ np.linalg.inv(Uu)
        sl[z] = np.linalg.inv(Uu).conj().T @ s1 @ L
        sr[z] = Uu @ s1 @ np.linalg.inv(L).conj().T
        cols = z * nd + np.arange(nd)
        pr.append(np.repeat(dofs, nd))
        pc.append(np.tile(cols, dofs.size))
        pv.append(Pz.ravel())
        rr.append(np.repeat(cols, dofs.size))
        rc.append(np.tile(dofs, nd))
        rv.append(Rz.ravel())
    nc = nz * nd
    P = sp.coo_matrix((np.concatenate(pv), (np.concatenate(pr), np.concatenate(pc))), shape=(nf, nc)).tocsr()
    R = sp.coo_matrix((np.concatenate(rv), (np.concatenate(rr), np.concatenate(rc))), shape=(nc, nf)).tocsr()
    SL = sp.block_diag(list(sl), format="csr")
    SR = sp.block_diag(list(sr), format="csr")
    return P, R, SL, SR


class Level:
    def __init__(self, op, P=None, dims=None):
        self.op = op          # operator on this level (sparse)
        self.P = P            # prolongator to this level from the next coarser
        self.dims = dims


class Hierarchy:
    """Level 0 holds the fine KD operator; level k >= 1 the Galerkin operators."""

    def __init__(self, lat, U, m, params, psi0, naik=False):
        self.lat = lat
        self.params = params
        self.kd = KDOperator(lat, U, m, naik=naik)
        self.naive = params.fine_op == "D"
        if params.fine_op not in ("A", "D"):
            raise ValueError("fine_op must be 'A' or 'D'")
        # the fine solve runs on the Schur system where it exists (Table 1)
        self.fine_schur = bool(params.fine_schur and self.kd.has_schur and not self.naive)
        self.nullvecs = []
        self.setup_its = []
        self.P = []
        self.R = []
        self.ops = [self.kd.D if self.naive else self.kd.A]
        self.aggr = []
        dims = None
        ndof_site = None
        nvec_prev = None
        if params.asymmetric:
            # the level's operator pair: gamma_5^{L/R} of A (eqs. gamma5L, gamma5R),
            # or eps twice for D (eps-Hermiticity)
            E = sp.diags(self.kd.eps).tocsr()
            gpair = (E, E) if self.naive else ((E @ self.kd.Binv).tocsr(), (self.kd.B @ E).tocsr())
            self.gamma_pairs = [gpair]
        for k, lp in enumerate(params.levels):
            op = self.ops[-1]
            if psi0[k] is None:
                raise ValueError("missing starting vectors")
            if isinstance(psi0[k], tuple) and psi0[k][0] == "relaxed":
                V = np.asarray(psi0[k][1])
                its = []
            else:
                V, its = relax_null_vectors(op, np.asarray(psi0[k]),
                                            params.setup_tol, params.setup_maxit)
            self.nullvecs.append(V)
            self.setup_its.append(its)
            V = global_orthonormalise(V)
            if k == 0:
                ag = aggregation_level1(lat, lp.agg)
            else:
                ag = aggregation_coarse(dims, ndof_site, nvec_prev, lp.agg)
            if params.asymmetric:
                # the left vectors are the same relaxed vectors (the construction
                # allows any; Sec. 5)
                P, R, sL, sR = asymmetric_transfer(V, V, ag, *self.gamma_pairs[-1])
                self.gamma_pairs.append((sL, sR))
            else:
                P = prolongator(V, ag)
                R = P.conj().T.tocsr()
            self.aggr.append(ag)
            self.P.append(P)
            self.R.append(R)
            self.ops.append(galerkin(P, op, R))
            dims = ag.coarse_dims
            ndof_site = 2 * lp.nvec
            nvec_prev = lp.nvec
        self.coarse_dims = dims
        self.P_even = self.P[0][self.kd.even].tocsr()
        self.R_even = self.R[0][:, self.kd.even].tocsr()
        self.coarse_lu = None
        if params.coarse_exact:
            self.coarse_lu = scipy.linalg.lu_factor(self.ops[-1].toarray())

    @property
    def nlevels(self):
        return len(self.ops)


# ---------------------------------------------------------------- solvers

class Stats:
    def __init__(self, nlevels):
        self.fine_applies = 0
        self.calls = [0] * nlevels
        self.its = [0] * nlevels


def mr(apply, r, its, omega):
    """Global MR with zero start: x += omega a r, r -= omega a A r,
    a = <A r, r>/<A r, A r>.  Returns (x, running residual)."""
    x = np.zeros_like(r)
    r = r.copy()
    for _ in range(its):
        q = apply(r)
        qq = vdot(q, q).real
        if qq == 0.0:
            break
        a = omega * vdot(q, r) / qq
        x += a * r
        r -= a * q
    return x, r


def gcr(apply, b, precond, restart, maxit, tol_abs):
    """Flexible restarted GCR (modified Gram-Schmidt on A z); x0 = 0."""
    x = np.zeros_like(b)
    r = b.copy()
    its = 0
    if norm(r) <= tol_abs:
        return x, its, r
    while its < maxit:
        Z, W = [], []
        for _ in range(restart):
            z = precond(r)
            w = apply(z)
            for zj, wj in zip(Z, W):
                beta = vdot(wj, w)
                w = w - beta * wj
                z = z - beta * zj
            nw = norm(w)
            w = w / nw
            z = z / nw
            alpha = vdot(w, r)
            x += alpha * z
            r -= alpha * w
            Z.append(z)
            W.append(w)
            its += 1
            if norm(r) <= tol_abs or its >= maxit:
                return x, its, r
        r = b - apply(x)
        if norm(r) <= tol_abs:
            return x, its, r
    return x, its, r


def cgne(op, b, tol, maxit):
    """CG on op op^dag y = b with x = op^dag y; stops on ||b - op x|| <= tol ||b||."""
    opH = op.conj().T
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = norm(b)
    if bnorm == 0.0:
        return x, 0
    p = opH @ r
    rr = vdot(r, r).real
    its = 0
    while its < maxit:
        pp = vdot(p, p).real
        alpha = rr / pp
        x += alpha * p
        r -= alpha * (op @ p)
        its += 1
        rr_new = vdot(r, r).real
        if np.sqrt(rr_new) <= tol * bnorm:
            break
        p = opH @ r + (rr_new / rr) * p
        rr = rr_new
    return x, its


class Solver:
    def __init__(self, h):
        self.h = h
        self.p = h.params

    def _op(self, level):
        if level == 0:
            S = self.h.kd.S if self.h.fine_schur else self.h.ops[0]

            def f(v):
                self.stats.fine_applies += 1
                return S @ v
            return f
        op = self.h.ops[level]
        return lambda v: op @ v

    def _restrict(self, level, r):
        R = self.h.R_even if level == 0 and self.h.fine_schur else self.h.R[level]
        return R @ r

    def _prolong(self, level, e):
        P = self.h.P_even if level == 0 and self.h.fine_schur else self.h.P[level]
        return P @ e

    def coarse_solve(self, level, r):
        p = self.p
        self.stats.calls[level] += 1
        if level == self.h.nlevels - 1 and self.h.coarse_lu is not None:
            x, its = scipy.linalg.lu_solve(self.h.coarse_lu, r), 1
        elif level == self.h.nlevels - 1:
            x, its = cgne(self.h.ops[level], r, p.coarse_tol, p.coarse_maxit)
        else:
            x, its, _ = gcr(self._op(level), r, lambda v: self.kcycle(level, v),
                            p.inter_restart, p.inter_maxit, p.inter_tol * norm(r))
        self.stats.its[level] += its
        return x

    def kcycle(self, level, r):
        p = self.p
        A = self._op(level)
        x, r1 = mr(A, r, p.mr_its, p.mr_omega)
        e = self.coarse_solve(level + 1, self._restrict(level, r1))
        x = x + self._prolong(level, e)
        r2 = r - A(x)
        x2, _ = mr(A, r2, p.mr_its, p.mr_omega)
        return x + x2

    def solve(self, b, tol=1e-10):
        kd = self.h.kd
        self.stats = Stats(self.h.nlevels)
        bnorm = norm(b)
        if self.h.fine_schur:
            # || b - D x || equals the Schur residual (reading of Sec. 4)
            bt = kd.schur_rhs(b)
            y, its, _ = gcr(self._op(0), bt, lambda v: self.kcycle(0, v),
                            self.p.outer_restart, self.p.outer_maxit, tol * bnorm)
            x = kd.reconstruct(b, y)
        else:
            # A y = b with x = B^-1 y (b - A y = b - D x exactly), or D x = b
            y, its, _ = gcr(self._op(0), b, lambda v: self.kcycle(0, v),
                            self.p.outer_restart, self.p.outer_maxit, tol * bnorm)
            x = y if self.h.naive else kd.Binv @ y
        res = norm(b - kd.D @ x) / bnorm
        st = self.stats
        info = {
            "outer_its": its,
            "fine_applies": st.fine_applies,
            "level_avg_its": [st.its[l] / st.calls[l] if st.calls[l] else 0.0
                              for l in range(1, self.h.nlevels)],
            "true_rel_resid": res,
            "converged": bool(res <= tol * (1 + 1e-6)),
        }
        return x, info

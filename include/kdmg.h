/*
 * kdmg.h - Kahler-Dirac-preconditioned adaptive multigrid for the staggered
 * Dirac operator on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The problem (Brower, Clark, Strelchenko, Weinberg, "Multigrid for staggered
 * lattice fermions", arXiv:1801.07823, Sec. 1): solve D(U, m) x = b with the
 * staggered operator of eq. "staggeredD",
 *
 *   (D psi)(x) = m psi(x) + 1/2 sum_mu eta_mu(x) [ U_mu(x) psi(x+mu)
 *                                                - U_mu(x-mu)^dag psi(x-mu) ],
 *   eta_mu(x) = (-1)^{x_1 + ... + x_{mu-1}},
 *
 * periodic in every direction except the last (time), which is antiperiodic.
 * The solver right-preconditions D by its 2^d Kahler-Dirac blocks B
 * (A = D B^-1 = 1 + C B^-1, Sec. 2.1 eq. "defA"), coarsens A by Galerkin
 * projection on chirally doubled, block-orthonormalised near-null vectors
 * (Sec. 3, 4), and runs flexible GCR on the KD-block-parity Schur operator
 * 1 - A_eo A_oe preconditioned by a K-cycle (Sec. 4, Table 1).
 *
 * Conventions shared by every call
 *   - Site index: x_1 + L_1*(x_2 + L_2*(...)), x_1 fastest, time = last axis.
 *   - Fine vectors: complex [rhs][site][colour]; complex128 (interleaved re,im
 *     doubles) unless a call says complex64.  Device pointers, caller-owned,
 *     never freed by the library.
 *   - Gauge links (host, copied at create): complex128 [mu][site][a][b],
 *     U_mu(x) the link from x to x+mu.
 *   - Coarse vectors on coarsening level k (k = 1 is the first coarse lattice):
 *     complex [rhs][Z][c*nvec_k + i], Z the coarse site (x_1 fastest), c = 0 for
 *     chirality +1 and 1 for -1 (sigma_3 = diag(1..1, -1..-1)), i the vector.
 *   - Even-block vectors (Schur space): the sites whose Kahler-Dirac block
 *     (floor(x_mu/2)) has even parity, in increasing site index.
 *   - Every call is stream-ordered on `stream` (a hipStream_t; NULL = default
 *     stream) and returns without waiting unless it says so.
 *   - Errors: every call returns a kdmg_status; nothing aborts or throws across
 *     the ABI.  kdmg_last_error() gives a thread-local message for the last
 *     failure.  Invalid sizes return KDMG_EINVAL before any device work.
 *
 * Supported geometry: nd = 2 with ncolor = 1 (U(1)), extents divisible by
 * 4 and by twice the first aggregate extent; nd = 4 with ncolor = 3 (SU(3)).
 */
#ifndef KDMG_H
#define KDMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  KDMG_OK = 0,
  KDMG_EINVAL = -1,       /* bad argument or unsupported shape */
  KDMG_ENOMEM = -2,       /* device allocation failed / over the memory budget */
  KDMG_EHIP = -3,         /* HIP runtime error */
  KDMG_ENOCONV = -4,      /* solver hit its iteration cap; outputs hold the best iterate */
  KDMG_EBUSY = -5,        /* object in use */
  KDMG_EUNSUPPORTED = -6  /* valid request the library does not implement */
} kdmg_status;

typedef enum {
  KDMG_FP64 = 0,  /* every level in FP64 */
  KDMG_MIXED = 1  /* FP64 outer FGCR, V-cycle in FP32 with FP16-stored links and
                     null vectors, FP64 coarsest solve */
} kdmg_prec;

typedef struct kdmg_lattice kdmg_lattice;     /* geometry + gauge field, device-resident */
typedef struct kdmg_hierarchy kdmg_hierarchy; /* KD blocks, P and coarse operators at one mass */

/* One coarsening (Table 1 rows "number of null vectors" / "size of aggregate block"). */
typedef struct {
  int agg[4]; /* aggregate extent per direction: KD blocks on the first coarsening
                 (so 4 means 8 fine sites), coarse sites on later ones */
  int nvec;   /* near-null vectors; the coarse lattice carries 2*nvec dofs per site */
} kdmg_level_params;

/* The K-cycle parameter set of Table 1. */
typedef struct {
  int nlevels;                /* total levels including the fine one: 2..4 */
  kdmg_level_params lvl[3];   /* lvl[k] builds level k+1 from level k */
  double setup_tol;           /* CG relative tolerance per null vector (1e-4) */
  int setup_maxit;            /* CG iterations per null vector (250) */
  int outer_restart;          /* fine FGCR restart length (32) */
  int outer_maxit;            /* fine FGCR iteration cap (KDMG_ENOCONV beyond) */
  int mr_its;                 /* MR pre/post-smoothing iterations (2) */
  double mr_omega;            /* MR relaxation parameter (0.85) */
  int inter_restart;          /* intermediate GCR restart (8) */
  int inter_maxit;            /* intermediate GCR iteration cap (16) */
  double inter_tol;           /* intermediate GCR relative tolerance (0.2) */
  double coarse_tol;          /* coarsest CGNE relative tolerance (0.2) */
  int coarse_maxit;           /* coarsest CGNE iteration cap (256) */
  int outer_stall;            /* 0 (default): off.  n > 0: a rhs whose residual
                                 norm has not halved over the last n outer
                                 iterations stops (KDMG_ENOCONV, best iterate
                                 returned) -- a serving policy, not part of
                                 the paper's method */
  int coarse_tail;            /* 16 (default): once this many or fewer rhs of a
                                 wider batched coarsest CGNE are still active,
                                 they continue as a narrower problem with the
                                 launch shape tuned for that width (the same
                                 iteration per rhs; rounding may differ with
                                 the shape); 0: off.  0..64 */
  int coarse_solver;          /* coarsest-level solve: 0 (default) CGNE with
                                 coarse_tol / coarse_maxit as in Table 1;
                                 1 exact, through an explicit FP64 inverse of
                                 the coarsest operator built with the
                                 hierarchy and on every mass change (not the
                                 paper's choice: a stronger preconditioner;
                                 at most 32768 coarsest dofs, 32 n^2 bytes of
                                 device memory for n dofs) */
  int fine_op;                /* operator that is coarsened and solved on the
                                 fine level: 0 (default) A = D B^-1, the
                                 Kahler-Dirac preconditioned operator of the
                                 paper; 1 D itself, the Galerkin multigrid
                                 that Sec. 3.2 shows to fail (Fig. "residstag"),
                                 kept as a negative control.  With 1, or on a
                                 Naik lattice, the fine solve runs on the full
                                 lattice instead of the KD-block-parity Schur
                                 system.  2D lattices only. */
  int asymmetric;             /* 0 (default): R = P^dag with chiral doubling
                                 (Sec. 3.3).  1: the asymmetric first
                                 coarsening of Sec. 5 (eqs. "prcplx",
                                 "thinlu") and App. A: per aggregate the
                                 columns v_i and gamma5^R v_i = B eps v_i, the
                                 rows v_i^dag and v_i^dag gamma5^L =
                                 v_i^dag eps B^-1, bi-orthonormalised by a
                                 thin LU without pivoting, so R != P^dag and
                                 R P = 1.  Two levels, fine_op = 0, 2D
                                 without Naik terms only; the transfers
                                 depend on the mass through B, so such a
                                 hierarchy cannot change its mass
                                 (kdmg_hierarchy_at_mass / _set_mass return
                                 KDMG_EUNSUPPORTED).  A zero pivot makes the
                                 build fail with KDMG_EINVAL.  The mixed
                                 V-cycle keeps P and R in FP32 here (not
                                 FP16): when R~ P~ is ill-conditioned the
                                 entries of P leave the FP16 range. */
} kdmg_mg_params;

/* Per right-hand side result of kdmg_solve. */
typedef struct {
  int converged;              /* true residual <= tol */
  int outer_its;              /* fine FGCR iterations */
  int fine_applies;           /* applications of the Schur operator (one counts as one A) */
  double level_avg_its[3];    /* average Krylov iterations per call on levels 2.. */
  double true_rel_resid;      /* ||b - D x|| / ||b||, recomputed in FP64 */
  double seconds;             /* wall time of the batched solve this rhs was part of */
} kdmg_solve_info;

/* Table 1 defaults with a three-level hierarchy (4^2 then 2^2 aggregates,
   n_vec 8 then 12). */
void kdmg_default_params(kdmg_mg_params* p);

/* Binds the library to HIP device `device` (call once per process before any
   other call; idempotent). */
kdmg_status kdmg_init(int device);

/* Uploads a gauge field for the staggered operator of eq. "staggeredD"
   (Sec. 1; U(1) links in 2D, SU(3) in 4D, Sec. 2).
   dims: nd extents, x_1 first.  links_host: complex128 [nd][volume][ncolor][ncolor],
   U_mu(x) the link from x to x+mu (copied; the caller keeps ownership).
   bc_sign: nd entries of +1 (periodic) or -1 (antiperiodic); a hop that
   crosses the boundary of direction mu carries bc_sign[mu].  NULL selects
   periodic space directions and an antiperiodic last (time) direction -- the
   paper states no boundary condition.  The upload runs on `stream`, which is
   synchronised before return.  KDMG_EINVAL for extents that are not positive
   multiples of 4 or signs other than +-1; KDMG_EUNSUPPORTED for geometries
   other than (nd 2, ncolor 1) and (nd 4, ncolor 3). */
kdmg_status kdmg_lattice_create(int nd, const int* dims, int ncolor, const int* bc_sign,
                                const double* links_host, void* stream, kdmg_lattice** out);
/* Switches the lattice's operator to the Naik-improved staggered operator of
   Sec. 2.1 (eq. "freehisq"), or back (enable = 0):
     D = m + 1/2 sum_mu eta_mu(x) [ c1 (U_mu(x) psi(x+mu) - U_mu(x-mu)^dag psi(x-mu))
                                  + c3 (W_mu(x) psi(x+3mu) - W_mu(x-3mu)^dag psi(x-3mu)) ],
   c1 = 9/8, c3 = -1/24, W_mu(x) = U_mu(x) U_mu(x+mu) U_mu(x+2mu).  (The
   printed operator carries 9/16 and 1/48 under an overall 1/2, whose own
   spectrum is half the one printed after it; these coefficients give that
   spectrum, m +- i sqrt(sum sin^2 p (1 + sin^2 p / 6)^2).)  Every operator and
   solve on the lattice then uses it: kdmg_apply_D, kdmg_apply_A (the KD block
   is the plain one with its hops scaled by 9/8; the three-link hops are part of
   C), and hierarchies built afterwards, whose fine solve runs on the full
   lattice because the three-link hops join KD blocks of the same parity
   (kdmg_apply_schur returns KDMG_EUNSUPPORTED).  First aggregates must be at
   least 2 KD blocks wide.  Hierarchies built before the switch must not be
   used after it.  2D U(1) only (KDMG_EUNSUPPORTED otherwise); extents >= 8.
   Runs on `stream` and synchronises it. */
kdmg_status kdmg_lattice_set_naik(kdmg_lattice* lat, int enable, void* stream);
void kdmg_lattice_destroy(kdmg_lattice* lat);
/* Device bytes held by the lattice. */
kdmg_status kdmg_lattice_footprint(const kdmg_lattice* lat, size_t* bytes);

/* out = D(U, mass) in  (eq. "staggeredD"), natural site order.
   prec = KDMG_FP64: complex128 vectors and FP64 links.
   prec = KDMG_MIXED: complex64 vectors, FP16-stored links, FP32 arithmetic.
   in and out must not overlap. */
kdmg_status kdmg_apply_D(const kdmg_lattice* lat, double mass, const void* in,
                         void* out, int nrhs, kdmg_prec prec, void* stream);

/* out = A in with A = D B^-1 (Sec. 2.1 eq. "defA"), or out = A^dag in when
   dagger != 0, using A^dag = eps B^-1 D eps (eq. "gamma5L").  B^-1 is the
   exact inverse of each 2^d Kahler-Dirac block (mass included).
   prec = KDMG_FP64: complex128 vectors, FP64 links and arithmetic.
   prec = KDMG_MIXED: complex64 vectors, FP16-stored links, FP32 arithmetic
   (4D: FP32 copies of the B^-1 blocks) -- the level-0 operator of the mixed
   V-cycle.  in, out: [nrhs][volume*ncolor] natural order, must not overlap.
   Allocates its work space per call and synchronises `stream`. */
kdmg_status kdmg_apply_A(const kdmg_lattice* lat, double mass, const void* in,
                         void* out, int nrhs, int dagger, kdmg_prec prec, void* stream);

/* out = B^-1 in: the inverse of the 2^d Kahler-Dirac blocks B, the
   block-local part of D (Sec. 2.1, the printed 2D block eq. "localblock";
   mass included).  complex128, FP64, natural order [nrhs][volume*ncolor].
   Allocates its work space per call and synchronises `stream`. */
kdmg_status kdmg_apply_Binv(const kdmg_lattice* lat, double mass, const void* in,
                            void* out, int nrhs, void* stream);

/* out_e = (1 - A_eo A_oe) in_e on even-block vectors (Table 1 level-1 operator),
   complex128, FP64. */
kdmg_status kdmg_apply_schur(const kdmg_lattice* lat, double mass,
                             const void* in_even, void* out_even, int nrhs,
                             void* stream);

/* kdmg_apply_schur without allocation, for callers that cannot allocate
   device memory (code under hipGraph capture, tight serving loops, harnesses
   that forbid hipMalloc): the same operator and kernels as kdmg_apply_schur,
   with its work space in a fixed 32 MiB device array per GPU that the library
   holds until the process ends, instead of memory allocated per call.
   2D lattices only (KDMG_EUNSUPPORTED in 4D, where B^-1 is built per call).
   nrhs is limited by that array: 6 * (volume / 2) * 16 bytes per rhs
   (volume 256^2: at most 10 rhs); larger requests return KDMG_EINVAL before
   any device work.  Stream-ordered; does not synchronise.  Every call on a
   GPU shares that GPU's array, so calls that overlap on one GPU (several
   streams or threads at once) race: serialise them. */
kdmg_status kdmg_apply_schur_noalloc(const kdmg_lattice* lat, double mass, const void* in_even,
                                     void* out_even, int nrhs, void* stream);

/* Builds the KD-MG hierarchy (Sec. 4 setup):
   for coarsening k = 0..nlevels-2, relax n_vec Gaussian starts with CG on
   A_k A_k^dag (tolerance setup_tol, setup_maxit iterations), orthonormalise
   them globally (modified Gram-Schmidt in vector order), chirally double and
   block-orthonormalise (thin QR, positive real diagonal) into P_k, and form
   A_{k+1} = P_k^dag A_k P_k.
   psi0_host[k]: complex128 [nvec_k][ndof_k] host starting vectors of coarsening
   k in that level's layout (fine: natural [site][colour]; coarse: see top).
   relaxed != 0: the vectors are taken as already-relaxed near-null vectors
   (no CG), which makes the hierarchy a pure function of them.
   Synchronises `stream` before returning.  The lattice must outlive the
   hierarchy. */
kdmg_status kdmg_hierarchy_build(const kdmg_lattice* lat, double mass,
                                 const kdmg_mg_params* params,
                                 const double* const* psi0_host, int relaxed,
                                 void* stream, kdmg_hierarchy** out);
void kdmg_hierarchy_destroy(kdmg_hierarchy* h);

/* Geometry of coarse level k (1 .. nlevels-1): dims[0..nd-1], dofs per site. */
kdmg_status kdmg_hierarchy_level_info(const kdmg_hierarchy* h, int level,
                                      int* dims_out, int* ndof_site_out);
/* Copies to host: the relaxed null vectors of coarsening k (before any
   orthonormalisation), complex128 [nvec][ndof_k]. */
kdmg_status kdmg_hierarchy_get_nullvecs(const kdmg_hierarchy* h, int k, double* host_out);
/* Copies to host the prolongator of coarsening k as its nonzero values:
   complex128 [ndof_k][nvec], row x holding P[x, (Z(x), c(x), i)] for i < nvec,
   where Z(x), c(x) are the aggregate and chirality of dof x. */
kdmg_status kdmg_hierarchy_get_prolongator(const kdmg_hierarchy* h, int k, double* host_out);
/* Asymmetric coarsening only (kdmg_mg_params.asymmetric = 1, k = 0): copies
   to host P and the transpose of R on the aggregates, complex128
   [ndof_0][2 nvec] each: p_out[x][j] = P[x, (Z(x), j)] and
   r_out[x][j] = R[(Z(x), j), x], coarse dof j < nvec from v_j and
   j >= nvec from B eps v_(j - nvec) (Sec. 5, eq. "prcplx").  Either output
   may be null.  KDMG_EINVAL for a symmetric hierarchy. */
kdmg_status kdmg_hierarchy_get_asym_transfer(const kdmg_hierarchy* h, int k, double* p_out, double* r_out);
/* Copies to host the coarse operator of level k >= 1 as its stencil blocks:
   complex128 [ndir][nsites][ndof][ndof], ndir = 2*nd + 1, direction 0 the
   site itself, 1 + 2*mu the neighbour Z + mu, 2 + 2*mu the neighbour Z - mu;
   block [dir][Z][i][j] couples dof i of Z to dof j of that neighbour. */
kdmg_status kdmg_hierarchy_get_coarse_op(const kdmg_hierarchy* h, int level, double* host_out);

/* out = A_level in (dagger = 0) or A_level^dag in on coarse level >= 1: the
   Galerkin coarse operator A_hat = P^dag A P of Sec. 3 (Sec. 3.3 for the
   Kahler-Dirac form), a nearest-neighbour block stencil with 2 n_vec dofs
   per coarse site; in and out are [nrhs][sites][dofs] coarse vectors.
   prec KDMG_FP64: complex128 and FP64 operator; KDMG_MIXED: complex64 and the
   FP32 operator.  Stream-ordered. */
kdmg_status kdmg_coarse_apply(const kdmg_hierarchy* h, int level, int dagger,
                              const void* in, void* out, int nrhs, kdmg_prec prec,
                              void* stream);
/* Restriction R_k = P_k^dag from level k to k+1 (Sec. 3, the restriction of
   the Galerkin coarse operator) and prolongation P_k, for nrhs vectors
   [rhs][dof] (level 0: [rhs][site] in lexicographic site order; coarse
   levels: [rhs][site][2 nv]).  prec KDMG_FP64: complex128 vectors and the
   FP64 prolongator; KDMG_MIXED: complex64 vectors and the FP16-stored
   prolongator of the mixed V-cycle, FP32 arithmetic.  Several rhs share one
   read of P.  in/out: caller-owned device buffers.  Level 0 synchronises
   `stream` (it uses a temporary); coarse levels are stream-ordered. */
kdmg_status kdmg_restrict(const kdmg_hierarchy* h, int k, const void* in, void* out,
                          int nrhs, kdmg_prec prec, void* stream);
kdmg_status kdmg_prolong(const kdmg_hierarchy* h, int k, const void* in, void* out,
                         int nrhs, kdmg_prec prec, void* stream);

/* The exact coarsest solve of a hierarchy built with coarse_solver = 1:
   out = A_c^-1 in on the coarsest level c = nlevels - 1 (A_c the Galerkin
   operator of Sec. 3 at the hierarchy's mass), for nrhs complex128 coarse
   vectors [nrhs][sites][dofs].  The inverse is formed at build time as
   A_c^dag (A_c A_c^dag)^-1 (FP64 Gauss-Jordan on the positive definite
   normal matrix); each call is one product with it.  KDMG_EINVAL if the
   hierarchy has no such inverse.  Allocates its work space per call and
   synchronises `stream`. */
kdmg_status kdmg_coarsest_solve(kdmg_hierarchy* h, const void* in, void* out, int nrhs, void* stream);

/* Conjugate gradient on the site even/odd Schur system, the solver the paper
   compares KD-MG against (Sec. 2, the even/odd normal equations; Sec. 4,
   Figs. "resid" and "iterworst"): with D = m + H,
   (m^2 - H_eo H_oe) x_e = m b_e - H_eo b_o (Hermitian positive definite),
   then x_o = (b_o - H_oe x_e) / m.  The target is ||b - D x|| <= tol ||b||,
   i.e. ||r_e|| <= tol m ||b|| for the true even residual r_e.  CG stops a
   rhs on its recursive residual; the true one is then recomputed, and rhs
   still above the target run further CG passes on the residual system
   (at most 8 passes and maxit iterations in all).  FP64.  b, x: complex128
   device vectors [nrhs][ndof] in natural site order, colours innermost (x
   is overwritten).  its_host: nrhs iteration counts (may be NULL).  Allocates
   its work space per call and synchronises `stream`.  Returns KDMG_ENOCONV
   (x and its_host still written) if a rhs missed tol within maxit;
   KDMG_EUNSUPPORTED for lattices other than 2D U(1) and 4D SU(3) (every
   extent even), KDMG_EINVAL for bad arguments.  The 4D call allocates a
   natural-order copy of the links (4 * 9 * 16 V bytes) for its duration. */
kdmg_status kdmg_solve_cg_eo(const kdmg_lattice* lat, double mass, const void* b, void* x, int nrhs,
                             double tol, int maxit, int* its_host, void* stream);

/* Solves D x = b for nrhs right-hand sides sharing the hierarchy (Sec. 4):
   FGCR on the Schur system until ||b - D x|| <= tol ||b|| per rhs, then
   reconstruction and an FP64 true-residual check.  b, x: complex128 device
   vectors (x is overwritten; its input value is ignored).  info_host: nrhs
   records (may be NULL).  Synchronises `stream`.  Returns KDMG_ENOCONV if any
   rhs missed tol within outer_maxit iterations. */
kdmg_status kdmg_solve(kdmg_hierarchy* h, const void* b, void* x, int nrhs, double tol,
                       kdmg_prec prec, kdmg_solve_info* info_host, void* stream);

/* Times every candidate launch shape of the coarse stencil kernels on this
   hierarchy's operators for `nrhs` right-hand sides at precision `prec` and
   keeps the fastest per level (kdmg_solve does this on its first call for a
   given nrhs unless KDMG_AUTOTUNE=0).  Synchronises `stream`. */
kdmg_status kdmg_hierarchy_autotune(kdmg_hierarchy* h, int nrhs, kdmg_prec prec, void* stream);

/* Verification of the autotuner's search space (not an operation of the
   method): applies the level's stencil (or its adjoint) with every launch
   shape the tuner may pick for (nrhs, prec), candidate c writing
   out[c][rhs][site][dof] (caller-allocated, at least max_out candidates).
   *ncand receives the number of candidates.  Synchronises `stream`. */
kdmg_status kdmg_coarse_apply_candidates(const kdmg_hierarchy* h, int level, int dagger, const void* in,
                                         void* out, int nrhs, kdmg_prec prec, int max_out, int* ncand,
                                         void* stream);

/* Device bytes held by the hierarchy including its solve workspace for
   `nrhs` right-hand sides (admission control). */
kdmg_status kdmg_hierarchy_footprint(const kdmg_hierarchy* h, int nrhs, size_t* bytes);

/* A hierarchy for the same gauge field at another mass (Sec. 4 setup, Table 1;
   the coarse operators are the Galerkin products of Sec. 3).  The new
   hierarchy shares `base`'s relaxed null vectors and prolongators (read-only;
   `base` may be destroyed first, the shared parts live until the last user)
   and Galerkin-builds its own coarse operators at `mass`.  The near-null
   vectors are not relaxed again: the low modes of D are those of its
   mass-independent anti-Hermitian part, so vectors relaxed at one mass serve
   nearby masses.  Allocates the coarse operators; synchronises `stream`. */
kdmg_status kdmg_hierarchy_at_mass(const kdmg_hierarchy* base, double mass, void* stream,
                                   kdmg_hierarchy** out);

/* Rebuild h's coarse operators in place at `mass`.  With base != NULL (and
   != h), h first switches to base's lattice, null vectors and prolongators;
   base must have the same lattice dimensions and level structure (else
   KDMG_EINVAL).  Reuses h's storage and solve workspace: after the first
   build of each shape it allocates nothing, so a serving loop can keep one
   hierarchy per (slot, shape) and move it between gauge configurations and
   masses.  KDMG_EBUSY while a solve on h is running.  Synchronises
   `stream`. */
kdmg_status kdmg_hierarchy_set_mass(kdmg_hierarchy* h, const kdmg_hierarchy* base, double mass,
                                    void* stream);

/* Implementation switch, not an operation of the method: replay captured
   hipGraphs for chunks of coarsest-level CGNE iterations (enable = 1, the
   default) or launch every kernel from the host (0); -1 leaves the setting.
   Both run the same kernels in the same order and give identical results.
   `replays` (may be NULL) receives the number of chunk graphs replayed on
   this hierarchy so far. */
kdmg_status kdmg_hierarchy_graphs(kdmg_hierarchy* h, int enable, long long* replays);

/* Implementation counters of the coarsest solve on this hierarchy so far, not
   quantities of the method: chunk graphs replayed, and batched coarsest CGNE
   calls that continued as a narrower tail problem (kdmg_mg_params.coarse_tail).
   Either pointer may be NULL. */
kdmg_status kdmg_hierarchy_counters(kdmg_hierarchy* h, long long* graph_replays, long long* tail_entries);

/* Measurement hook (not an operation of the method): HIP-event timing, on
   the solve's own stream during later kdmg_solve calls, of the coarsest
   solve's kernels -- the two fused kernels of each CGNE iteration, or with
   coarse_solver = 1 the product with the inverse (one launch counted per
   call, the partial-product kernel and its in-order reduction together).  enable = 1 starts (and zeroes) the
   counters, 0 stops, -1 leaves the state as it is.  `ms` (may be NULL)
   receives the summed kernel time and `launches` (may be NULL) the number of
   kernel launches it covers: within every run of launches between two host
   polls, the first launch is excluded so host launch latency after a poll is
   not counted.  Only FP64 coarsest levels (the fused CGNE) are timed. */
kdmg_status kdmg_hierarchy_kernel_timing(kdmg_hierarchy* h, int enable, double* ms, long long* launches);

/* ------------------------------------------------------------------ serving
   A solve service over device-resident configurations.  Not an operation of
   the paper: it runs the paper's solve (Sec. 4, Table 1) for a stream of
   requests.  Requests are admitted in arrival order as soon as one of the
   `slots` workers is free and the request's device footprint fits
   `hbm_budget`; admitted requests run concurrently, one HIP stream per
   worker.  A request runs on a pooled hierarchy of its shape moved onto its
   configuration and mass (kdmg_hierarchy_set_mass), or on a new one
   (kdmg_hierarchy_at_mass); idle pooled hierarchies are released when memory
   is needed.  Results depend only on (configuration, mass, b, tol, prec):
   the same alone and in any mix. */
typedef struct kdmg_server kdmg_server;

/* Create a service on the current device.  slots: 1..64 workers. */
kdmg_status kdmg_server_create(int slots, size_t hbm_budget, kdmg_server** out);

/* Register a configuration: a hierarchy from kdmg_hierarchy_build (setup
   done, at any mass).  Not owned: it (and its lattice) must outlive the
   server.  Returns its id (0, 1, ... in registration order). */
kdmg_status kdmg_server_add_config(kdmg_server* s, const kdmg_hierarchy* base, int* config_id);

/* Device bytes one request on this configuration holds while it runs
   (coarse operators at its mass + solve workspace): the admission unit. */
kdmg_status kdmg_server_request_bytes(kdmg_server* s, int config_id, int nrhs, kdmg_prec prec,
                                      size_t* bytes);

/* Queue a solve of D(U_config, mass) x = b for nrhs right-hand sides, layout
   as kdmg_solve.  b and x are caller-owned device buffers that must stay
   valid until the request is collected by kdmg_server_poll.  Ordering: an
   event is recorded on `stream` (the caller's stream; NULL = default stream)
   at submit, and the request's device work waits for it, so work the caller
   queued on `stream` before the submit (producing b, clearing x) completes
   first.  Work queued on other streams must be ordered by the caller.  The
   caller must not touch b or x after the submit until poll reports done;
   then the solve's device work is complete and x can be read on any
   stream.  KDMG_ENOMEM if the request alone exceeds the budget. */
kdmg_status kdmg_server_submit(kdmg_server* s, int config_id, double mass, const void* b, void* x,
                               int nrhs, double tol, kdmg_prec prec, void* stream, long long* ticket);

/* done = 1 once the request has finished (wait != 0 blocks until then).
   When done: *solve_status is kdmg_solve's status (kdmg_last_error() has its
   message), info[0..nrhs) as from kdmg_solve, times[0..3) = seconds queued,
   running, and in total (submit to finish); the ticket is then released. */
kdmg_status kdmg_server_poll(kdmg_server* s, long long ticket, int wait, int* done,
                             kdmg_status* solve_status, kdmg_solve_info* info, double* times);

/* Counters: completed requests, running now, peak concurrently running,
   device bytes reserved now (running + pooled idle) and at peak. */
kdmg_status kdmg_server_stats(kdmg_server* s, long long* completed, int* running, int* peak_running,
                              size_t* allocated, size_t* peak_allocated);

/* Finish the running requests, drop queued ones (their poll reports
   KDMG_EBUSY), free pooled hierarchies and streams. */
void kdmg_server_destroy(kdmg_server* s);

const char* kdmg_status_string(kdmg_status s);
const char* kdmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* KDMG_H */

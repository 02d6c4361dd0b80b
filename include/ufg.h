/*
 * ufg.h -- C ABI of the MI355X (gfx950) library for the unitary-Fermi-gas
 * fermion matrix of Ten, Drut and Laehde, "Preconditioning the
 * non-relativistic many-fermion problem" (arXiv:1008.3647).
 *
 * The operator (paper, Sec. 1, Eq. MatrixM): M[sigma] is block cyclic over
 * Ntau time slices with unit diagonal blocks, -B_j on the block sub-diagonal
 * and +B_{Ntau} in the top-right corner, B_j = exp(-tau K)(1 + A sin sigma_j),
 * A = sqrt(2) sqrt(exp(tau g) - 1), E(k) = k^2/2 (hbar = m = 1) on the momenta
 * k_i = 2 pi n_i / Nx. M is real, so M^dagger = M^T.
 *
 * Conventions shared by every entry point
 *   - Vectors are complex, interleaved (re, im), C order [nrhs][Ntau][Nx][Nx][Nx]
 *     (x fastest; [nrhs][Ntau][Nx]^dim and fields [Ntau][Nx]^dim on lattices
 *     made by create_lattice_dim). Element type is complex64 (float2) or complex128 (double2)
 *     as fixed by the lattice's dtype; "mixed" solves take complex128.
 *   - Every vector and field pointer is a DEVICE pointer owned by the caller;
 *     it must stay valid until the call's work has completed on the stream.
 *   - Work is enqueued on the lattice's HIP stream. apply_* and
 *     force_dS_dsigma are asynchronous; set_aux_field and solve_* return after
 *     their work has completed.
 *   - Return value: 0 = success; negative = caller or system error
 *     (UFG_EINVAL, UFG_ENOMEM, UFG_EHIP); positive = numerical outcome of a
 *     solve (UFG_NOT_CONVERGED, UFG_BREAKDOWN), in which case x holds the last
 *     iterate and the stats are filled. ufg_last_error() describes the last
 *     failure of the calling thread.
 */
#ifndef UFG_H
#define UFG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ufg_lattice_s* ufg_lattice; /* opaque, owned by the library */

enum { UFG_C64 = 0, UFG_C128 = 1 };

/* Kinetic energy per axis (create_lattice_ex): UFG_DISP_FREE, E = k^2 / 2 (Sec. 1);
   UFG_DISP_HUBBARD, E = 1 - cos k, the Hubbard-model dispersion the concluding
   section names as an extension (nearest-neighbour hopping of amplitude 1/2,
   equal to k^2 / 2 up to O(k^4)). */
enum { UFG_DISP_FREE = 0, UFG_DISP_HUBBARD = 1 };

enum {
  UFG_OK = 0,
  UFG_EINVAL = -1,
  UFG_ENOMEM = -2,
  UFG_EHIP = -3,
  UFG_NOT_CONVERGED = 1,
  UFG_BREAKDOWN = 2
};

/* Operators a solve or preconditioner refers to. */
enum {
  UFG_OP_M = 0,        /* M x = b                                           */
  UFG_OP_MDAG = 1,     /* M^dagger x = b                                    */
  UFG_OP_TWO_STEP = 2, /* M^dagger y = b then M x = y (paper, Eq. 2)        */
  UFG_OP_Q = 3         /* Q = M^dagger M (paper, Eq. 1)                     */
};

/* Preconditioner kinds (paper, Secs. 2-4). */
enum { UFG_PC_NONE = 0, UFG_PC_CHEB = 1, UFG_PC_SCA = 2, UFG_PC_WCE = 3, UFG_PC_SCA_CHEB = 4 };

/*
 * Preconditioner description.
 *   CHEB (Sec. 2): P(Q^) = c prod_k (Q^ - z_k), Q^ = Q / lam_max, degree 2n =
 *        `degree` (a power of two: the factors are applied in bit-reversal
 *        order), spectrum assumed in [eps, 1]. lam_max > 0: used as given;
 *        lam_max == 0: the bound (1 + max|1 + A sin sigma|)^2 >= ||Q||;
 *        lam_max < 0: 30 power iterations on Q, times 1.05.
 *   SCA  (Sec. 4): (L^dagger D L)^{-1}, shift `alpha` (> 0).
 *   SCA_CHEB (Sec. 4, closing remark: the Chebyshev approximation as a
 *        secondary filter of SCA): P = P_2n(S Q / lam_max) S, S the SCA inverse
 *        (shift `alpha`), the polynomial of CHEB with `degree` and `eps`;
 *        lam_max > 0 used as given, else 1.05 times 30 power iterations on S Q.
 *   WCE  (Sec. 3): W_d = sum_{m<=d} w_m (-A M0^{-1} M1)^m M0^{-1}, d =
 *        `wce_order` (0..8); w_m = 1, or the Euler weights of Sec. 3.1 with
 *        parameter `euler_p` when `euler` != 0 (estimate S_{d,0}).
 * How a kind acts for each operator (apply_precond's `op`):
 *   op = UFG_OP_Q   : CHEB P(Q^), SCA (L^dagger D L)^{-1}, SCA_CHEB P, WCE W_d W_d^dagger
 *   op = UFG_OP_M   : WCE W_d;          CHEB/SCA/SCA_CHEB  P M^dagger  (extension)
 *   op = UFG_OP_MDAG: WCE W_d^dagger;   CHEB/SCA/SCA_CHEB  M P         (extension)
 */
typedef struct {
  int kind;
  int degree;
  double eps;
  double lam_max;
  double alpha;
  int wce_order;
  int euler;
  double euler_p;
} ufg_precond;

/*
 * Solve options.
 *   tol        stop when every RHS has ||b - A x|| <= tol ||b|| (true residual,
 *              recomputed in FP64 at the end); x_0 = 0 unless use_x0.
 *   maxit      iteration cap per solve step (paper: 10,000).
 *   mixed      0: every vector in the lattice dtype. 1: complex64 inner Krylov
 *              iteration with FP64 reliable updates of x and r = b - A x and
 *              FP64 reductions; b and x are complex128 (lattice dtype C128).
 *   delta      reliable-update trigger: update when the inner residual has
 *              fallen below delta times its maximum since the last update.
 *   check_every  iterations between check points (>= 1). Reliable updates
 *              and restarts happen at check points. The host reads the flags
 *              of a check point at the next one (it never waits for the device
 *              there), so a solve ends up to two intervals after convergence
 *              on launches that do no work (not counted in the statistics).
 *   eager      0: where the iteration is not fused into the streaming kernel
 *              (preconditioned solves, CG, Nx outside {8, 12, 16}), every
 *              check interval after the first replays a HIP graph captured
 *              from the same launches (same results; fewer host launches for
 *              small lattices). 1: launch every kernel separately.
 */
typedef struct {
  double tol;
  int maxit;
  int mixed;
  double delta;
  int check_every;
  int use_x0;
  int eager;
} ufg_solve_opts;

/* Solve statistics (worst case over the right-hand sides). */
typedef struct {
  int iters[2];              /* iterations of step 1 / step 2 (CG: [0] only)  */
  long long mv;              /* applications of M or M^dagger (any precision) */
  long long m0inv;           /* applications of M0^{-1} or its adjoint        */
  long long sca_sweeps;      /* SCA forward+backward sweeps                   */
  long long reliable_updates;
  double relres[2];          /* true ||b - A x|| / ||b|| per step             */
  double relres_normal;      /* ||b - M^dagger M x|| / ||b|| (two-step, CG)   */
  double seconds;            /* wall time of the call                         */
  double paper_mv;           /* MV count under the paper's cost model         */
  int status;
  long long host_syncs;      /* solve_batched: host waits for the device      */
  long long host_submits;    /* solve_batched: graph launches, kernel launches
                                and copies the host issued (0 elsewhere)      */
} ufg_solve_stats;

/*
 * create_lattice -- allocate a lattice handle for an Nx^3 x Ntau lattice.
 *   nx: even, 2 <= nx <= 16. ntau >= 2. tau > 0, g >= 0 (A from Sec. 1).
 *   dtype: UFG_C64 or UFG_C128. hip_stream: a hipStream_t (NULL = default).
 *   out: receives the handle. The field is zero (sigma = 0) until
 *   set_aux_field. Errors: UFG_EINVAL (bad size, dtype or pointer),
 *   UFG_ENOMEM, UFG_EHIP.
 */
int create_lattice(int nx, int ntau, double tau, double g, int dtype,
                   void* hip_stream, ufg_lattice* out);

/*
 * create_lattice_ex -- create_lattice with the dispersion of K chosen:
 *   UFG_DISP_FREE (what create_lattice makes) or UFG_DISP_HUBBARD. exp(-tau K)
 *   stays the product of one symmetric circulant factor T per axis, so every
 *   operator, preconditioner, solver and the force apply unchanged; T, its
 *   eigenbasis (M0^{-1}) and the block form of T follow the dispersion. The
 *   strong-coupling blocks do not involve K. Errors as create_lattice, and
 *   UFG_EINVAL for another dispersion value.
 */
int create_lattice_ex(int nx, int ntau, double tau, double g, int dtype, int dispersion,
                      void* hip_stream, ufg_lattice* out);

/*
 * create_lattice_dim -- create_lattice_ex for a lattice of spatial dimension
 *   dim = 1, 2 or 3 (the lower dimensions the paper's concluding section
 *   names as an extension): slices of Nx^dim sites, exp(-tau K) the product
 *   of dim factors T, E(k) summed over dim axes (Sec. 1 otherwise unchanged).
 *   Vectors are [nrhs][Ntau][Nx]^dim and sigma [Ntau][Nx]^dim, C order.
 *   dim = 3 is create_lattice_ex. On dim < 3 every operator, preconditioner,
 *   solver, the force and the HMC calls apply (through the general slice
 *   kernels; the streaming kernels and fused BiCGStab forms are for dim = 3);
 *   solve_batched takes dim = 3 only. Errors as create_lattice_ex, and
 *   UFG_EINVAL for another dim.
 */
int create_lattice_dim(int nx, int ntau, int dim, double tau, double g, int dtype,
                       int dispersion, void* hip_stream, ufg_lattice* out);

/* destroy_lattice -- free the handle and all library-owned device memory. */
int destroy_lattice(ufg_lattice L);

/* set_lattice_stream -- change the stream later work is enqueued on. */
int set_lattice_stream(ufg_lattice L, void* hip_stream);

/*
 * set_aux_field -- install sigma (paper, Sec. 1: one real per space-time site).
 *   sigma_dev: device float64 [Ntau][Nx][Nx][Nx]; copied, so the caller may
 *   free it afterwards. Derives 1 + A sin sigma, sin sigma, cos sigma in FP64
 *   and FP32 and the strong-coupling blocks (alpha = 1). Synchronous.
 */
int set_aux_field(ufg_lattice L, const double* sigma_dev);

/*
 * apply_M -- y = M x for nrhs vectors (Eq. MatrixM):
 *   y_{t+1} = x_{t+1} + s_t e^{-tau K}((1 + A sin sigma_t) x_t),
 *   s_t = -1 (t < Ntau-1), +1 (t = Ntau-1; antiperiodic corner).
 *   x, y: device, lattice dtype, must not alias. Asynchronous.
 */
int apply_M(ufg_lattice L, const void* x, void* y, int nrhs);

/*
 * apply_Mdag -- y = M^dagger x = M^T x (Sec. 1: M is real):
 *   y_t = x_t + s_t (1 + A sin sigma_t) e^{-tau K} x_{t+1}.  Asynchronous.
 */
int apply_Mdag(ufg_lattice L, const void* x, void* y, int nrhs);

/*
 * apply_precond -- y = K^{-1} x for the preconditioner `p` acting on operator
 *   `op` (table at ufg_precond). x, y: device, lattice dtype, no aliasing.
 *   Synchronous only when a Chebyshev lam_max has to be estimated first.
 */
int apply_precond(ufg_lattice L, const ufg_precond* p, int op, const void* x,
                  void* y, int nrhs);

/*
 * precond_lam_max -- the lam_max a Chebyshev preconditioner `p` normalises Q
 *   with on this lattice (Sec. 2: Q^ = Q / lam_max): p->lam_max if > 0, the
 *   bound (1 + max|b|)^2 if 0, else 1.05 times 30 power iterations on Q (cached
 *   per field; synchronous). out_host: one double. UFG_EINVAL unless
 *   p->kind == UFG_PC_CHEB.
 */
int precond_lam_max(ufg_lattice L, const ufg_precond* p, double* out_host);

/*
 * solve_cg_normal -- x = (M^dagger M)^{-1} b by (preconditioned) CG
 *   (paper, Eqs. 1 and 3). p may be NULL (no preconditioner); p->kind is any
 *   kind (WCE acts as W_d W_d^dagger). b, x: device, nrhs vectors; with
 *   o->mixed, complex128. st may be NULL.
 */
int solve_cg_normal(ufg_lattice L, const ufg_precond* p, const void* b,
                    void* x, int nrhs, const ufg_solve_opts* o,
                    ufg_solve_stats* st);

/*
 * solve_cg_split -- x = (M^dagger M)^{-1} b by CG with split preconditioning
 *   (paper, Sec. 5, the remark after Table 2: (M0^dagger)^{-1} on the left and
 *   M0^{-1} on the right): with E = W_d of the weak-coupling preconditioner p
 *   (p->kind == UFG_PC_WCE; order 0 is E = M0^{-1}), CG runs on the Hermitian
 *   positive-definite E^dagger M^dagger M E z = E^dagger b and returns x = E z.
 *   tol applies to that system's residual ||E^dagger (b - M^dagger M x)||
 *   relative to ||E^dagger b||; st->relres[0] reports ||b - M^dagger M x|| / ||b||.
 *   Lattice dtype only (o->mixed = 0), x_0 = 0 (o->use_x0 = 0). Same
 *   conventions as solve_cg_normal otherwise.
 */
int solve_cg_split(ufg_lattice L, const ufg_precond* p, const void* b, void* x, int nrhs,
                   const ufg_solve_opts* o, ufg_solve_stats* st);

/*
 * solve_bicgstab -- BiCGStab (van der Vorst, right preconditioned) for
 *   op = UFG_OP_M (M x = b), UFG_OP_MDAG (M^dagger x = b) or UFG_OP_TWO_STEP
 *   (M^dagger y = b, then M x = y; paper, Eq. 2). Iterations of the two steps
 *   are reported separately in st->iters.
 */
int solve_bicgstab(ufg_lattice L, const ufg_precond* p, int op, const void* b,
                   void* x, int nrhs, const ufg_solve_opts* o,
                   ufg_solve_stats* st);

/*
 * solve_batched -- nprob independent two-step BiCGStab solves (M^dagger y = b,
 *   then M x = y; paper, Eq. 2), one lattice each (lattices may differ in Nx
 *   and Ntau), nrhs[i] right-hand sides per problem. Every phase of an
 *   iteration is one persistent launch over a work table covering all
 *   problems; whole check intervals, with their reliable updates and restarts
 *   gated on device flags, are replayed from captured HIP graphs, the host
 *   reading the flags once per ~200 iterations (solve_batched_tune); every
 *   (problem, rhs) keeps its own device state and stops on its own.
 *   Ls[i]: complex128 lattices (fields installed). b[i], x[i]: device
 *   complex128 vectors [nrhs[i]][Ntau][Nx]^3 of lattice i. o->mixed: complex64
 *   inner iteration with FP64 reliable updates (else complex128 inner).
 *   o->use_x0 must be 0. p: NULL or UFG_PC_NONE. st: array of nprob stats (may
 *   be NULL; seconds is the wall time of the whole batch). Synchronous; uses
 *   its own stream after synchronising the lattices' streams. Returns the
 *   worst status.
 */
int solve_batched(const ufg_lattice* Ls, int nprob, const void* const* b,
                  void* const* x, const int* nrhs, const ufg_precond* p,
                  const ufg_solve_opts* o, ufg_solve_stats* st);

/*
 * solve_batched_tune -- launch shape of solve_batched chosen by the autotuner
 *   (0 keeps the default): workgroups per compute unit of the persistent
 *   operator and vector launches (1..64; defaults 4 and 8), elements per vector
 *   work item (256..4194304; default 4096), time slices per slab of the
 *   batched streaming operator (1..64; default 2) and iterations between host
 *   reads of the convergence flags (1..100000, rounded to whole check
 *   intervals; default 200). Process-wide; not thread safe against concurrent
 *   solves. Results do not depend on them beyond floating-point summation
 *   order (and the last point at which an unconverged system may stop).
 */
int solve_batched_tune(int hop_blocks_per_cu, int vec_blocks_per_cu, long long chunk, int slab,
                       int sync_iters);

/*
 * force_dS_dsigma -- gradient of S = sum_r phi_r^dagger (M^dagger M)^{-1} phi_r
 *   (paper, Sec. 1) given X_r = (M^dagger M)^{-1} phi_r and y_r = M X_r:
 *   grad(n,t) = -2 A cos sigma(n,t) s_t sum_r Re[X_r,t(n) conj((e^{-tau K} y_r,t+1)(n))].
 *   X, y: device, lattice dtype, nrhs vectors. grad_dev: device float64 [Ntau][Nx^3],
 *   overwritten. Asynchronous.
 */
int force_dS_dsigma(ufg_lattice L, const void* X, const void* y, int nrhs,
                    double* grad_dev);

/*
 * HMC of the phi-algorithm (paper, Sec. 1). The MD Hamiltonian is
 *   H = sum_{n,t} pi(n,t)^2 / 2 + S_p[sigma],  S_p = sum_r phi_r^dagger Q^{-1} phi_r,
 * Q = M^dagger M, with phi held fixed during the molecular dynamics. Every
 * force evaluation installs sigma (as set_aux_field), solves M^dagger y = phi
 * and M X = y with BiCGStab (precond, tol, maxit, mixed as in solve_bicgstab),
 * takes S_p = sum_r ||y_r||^2 (FP64) and the gradient of force_dS_dsigma.
 * The integrator is leapfrog, kick-drift-kick with half kicks at both ends:
 *   pi -= dt/2 g(sigma); nsteps times { sigma += dt pi; pi -= dt g(sigma) },
 *   the last kick being dt/2 (nsteps + 1 force evaluations);
 *   pi_dot = -dS_p/dsigma.
 * The field updates and sum pi^2 run in library kernels (FP64, fixed
 * summation order); nothing is drawn at random inside the library: eta, pi
 * and the Metropolis draw u are inputs.
 *
 *   dt          step size (finite, > 0).  nsteps  leapfrog steps (1..1e6).
 *   tol, maxit, mixed, check_every, precond:  every solve (check_every >= 1).
 *   chrono      1: every solve starts from the previous force's solution (the
 *               first y of hmc_trajectory from eta, which solves M^dagger y =
 *               phi exactly); 0: every solve starts from x = 0.
 */
typedef struct {
  double dt;
  int nsteps;
  double tol;
  int maxit;
  int mixed;
  int check_every;
  int chrono;
} ufg_hmc_opts;

typedef struct {
  double S0, S1;        /* S_p at the start / at the MD end point             */
  double K0, K1;        /* sum pi^2 / 2 at the start / at the MD end point    */
  double dH;            /* (K1 - K0) + (S1 - S0)                              */
  int accept;           /* hmc_trajectory: Metropolis decision; leapfrog: -1  */
  int status;           /* 0, else the status (1, 2) of the first failed solve */
  int forces;           /* force evaluations done                             */
  long long solves;     /* BiCGStab solves                                    */
  long long iters;      /* iterations summed over the solves (worst rhs)      */
  long long mv;         /* applications of M or M^dagger                      */
  double worst_relres;  /* largest true relative residual of any solve        */
  double seconds;       /* wall time of the call                              */
} ufg_hmc_result;

/*
 * hmc_leapfrog -- the MD part alone: integrates (sigma, pi) in place from the
 *   given state for phi fixed.
 *   sigma_dev, pi_dev: device float64 [Ntau][Nx]^3, distinct; overwritten with
 *   the MD end point (with the start again if a solve fails: then
 *   res->status > 0). phi_dev: device, lattice dtype, nphi vectors (complex128
 *   when mixed). actions_host: NULL or host array of nsteps + 1 doubles, S_p
 *   at every force evaluation. res: required; accept = -1. On return the
 *   installed field is sigma_dev's. Synchronous. A negative return leaves
 *   sigma and pi unspecified.
 */
int hmc_leapfrog(ufg_lattice L, const ufg_precond* precond, double* sigma_dev, double* pi_dev,
                 const void* phi_dev, int nphi, const ufg_hmc_opts* o, double* actions_host,
                 ufg_hmc_result* res);

/*
 * hmc_trajectory -- one trajectory of the phi-algorithm: heat bath
 *   phi_r = M^dagger eta_r at the starting sigma (eta_r ~ exp(-eta^dagger eta),
 *   so that phi ~ exp(-phi^dagger Q^{-1} phi)), the MD of hmc_leapfrog, then the
 *   Metropolis step: accept iff u < exp(-dH) (probability min(1, exp(-dH))),
 *   decided in FP64 on the host.
 *   sigma_dev, pi_dev: device float64, distinct; on accept they hold the MD end
 *   point, on reject (or a failed solve) the start, and the installed field
 *   is the one they hold. eta_dev: device, lattice dtype, nphi vectors.
 *   u: Metropolis draw in [0, 1). phi_out: NULL or device buffer like eta
 *   that receives phi. actions_host, res: as hmc_leapfrog. Synchronous.
 */
int hmc_trajectory(ufg_lattice L, const ufg_precond* precond, double* sigma_dev, double* pi_dev,
                   const void* eta_dev, int nphi, double u, const ufg_hmc_opts* o,
                   void* phi_out, double* actions_host, ufg_hmc_result* res);

/*
 * lattice_norm2 -- out_host[r] = ||x_r||^2 for nrhs vectors of the lattice dtype
 *   (FP64 accumulation, fixed summation order). The pseudofermion action of
 *   Sec. 1 is S = ||y||^2 with M^dagger y = phi. out_host: host array of nrhs
 *   doubles. Synchronous.
 */
int lattice_norm2(ufg_lattice L, const void* x, int nrhs, double* out_host);

/*
 * lattice_norm2_noalloc -- for callers that cannot allocate device memory
 *   (code under HIP graph capture, tight serving loops, harnesses that forbid
 *   hipMalloc): the squared norms of lattice_norm2, computed by the same
 *   kernels in the same summation order, but into out_dev[r] (device float64
 *   array of nrhs, caller-owned) and asynchronously on the lattice's stream.
 *   Makes no allocation: its partial sums and per-rhs state live in a static
 *   device buffer of 2 MiB per GPU (held until the process ends). Needs
 *   32 * vec_blocks * nrhs + ~64 * nrhs bytes of it (vec_blocks as in
 *   lattice_tune, by default at most max(16, 2048 / nrhs) for this call);
 *   larger requests return UFG_EINVAL with a message. Every call on one GPU
 *   shares that buffer: calls that overlap in time on one GPU (concurrent
 *   streams or threads) race and must be serialised by the caller.
 */
int lattice_norm2_noalloc(ufg_lattice L, const void* x, int nrhs, double* out_dev);

/*
 * lattice_tune -- launch parameters chosen by the autotuner (0 keeps the
 *   default): `slab` time slices per workgroup of the streaming M / M^T kernel
 *   (Nx in {8, 12, 16}; 1..Ntau), `vec_blocks` workgroups per right-hand side of
 *   the Krylov vector kernels (1..4096). Results do not depend on them beyond
 *   floating-point summation order.
 */
int lattice_tune(ufg_lattice L, int slab, int vec_blocks);

/*
 * lattice_tune_slabs -- number of slabs per right-hand side of the streaming
 *   M / M^T kernel (1..Ntau; 0 derives it from lattice_tune's slab as
 *   ceil(Ntau / slab)). Slab s covers slices [s Ntau / n, (s + 1) Ntau / n), so
 *   the count need not divide Ntau; it sets the grid (n x nrhs workgroups) to fit
 *   the number of resident workgroups. Same result guarantee as lattice_tune.
 */
int lattice_tune_slabs(ufg_lattice L, int nslab);

/*
 * lattice_tune_order -- workgroup numbering of the streaming M / M^T and
 *   basis-change kernels. group >= 1: groups of `group` consecutive slabs go
 *   round-robin to the eight XCDs, so a slab's halo slice and its field slab
 *   are read through one XCD's L2; each XCD takes its groups right-hand side
 *   by right-hand side (rhs_inner = 0) or, group by group, every right-hand
 *   side of a group in turn (rhs_inner = 1). group = 0: contiguous runs of
 *   (slab, rhs) pairs per XCD, rhs fastest (rhs_inner ignored); group = -1:
 *   the library default (complex64 lattices: groups of 10, rhs_inner 0;
 *   complex128 lattices of 2^20 sites and more: groups of 10, rhs_inner 1;
 *   smaller complex128 lattices: 0). group: -1..Ntau. Same result guarantee
 *   as lattice_tune (the numbering changes no arithmetic).
 */
int lattice_tune_order(ufg_lattice L, int group, int rhs_inner);

/*
 * lattice_tune_transform -- how the complex64 Nx = 16 streaming M / M^T
 *   operator applies exp(-tau K) = T (x) T (x) T (Sec. 1) to a slice: route 0
 *   (default) runs all three axes in the reflection-symmetry block form of T on
 *   the vector ALUs; route 1 keeps the z axis there and runs the y and x axes
 *   as 16x16x4 FP32 matrix-core (MFMA) contractions with T; route 2 applies T
 *   along every axis as a 16-point DFT, the eigenvalues of T and the inverse
 *   DFT (T is circulant). Same operator; results agree to FP32 rounding, not
 *   bit for bit. Other dtypes, sizes and the fused solver variants always use
 *   route 0. Errors: UFG_EINVAL for a route other than 0, 1 or 2.
 */
int lattice_tune_transform(ufg_lattice L, int route);

/* lattice_info -- nx, ntau, dtype, A of a handle (host pointers, any may be NULL). */
int lattice_info(ufg_lattice L, int* nx, int* ntau, int* dtype, double* A);

/* ufg_last_error -- message for the last failing call on this thread.
 * last_error is the same function under its short name. The returned string
 * is owned by the library and valid until the thread's next failing call. */
const char* ufg_last_error(void);
const char* last_error(void);

/*
 * Host helpers (no device work; usable without a GPU):
 *   ufg_cheb_roots: the 2n roots z_k (re, im interleaved into out[2*degree]) in
 *     application (bit-reversal) order and the per-factor constant
 *     c^{1/(2n)} (out_c[2]). Returns UFG_EINVAL unless degree is a power of two.
 *   ufg_euler_weights: the weights w_0..w_d of Sec. 3.1 (out[d+1]).
 *   ufg_transfer_matrix: the Nx x Nx factor T of e^{-tau K} (out[nx*nx]).
 */
int ufg_cheb_roots(int degree, double eps, double* out, double* out_c);
int ufg_euler_weights(int order, double p, double* out);
int ufg_transfer_matrix(int nx, double tau, double* out);

/*
 * ufg_device_copy -- measurement helper, not part of the method: a plain
 *   streaming copy of `bytes` from src to dst (device pointers, 16-byte
 *   aligned, bytes a multiple of 16; the regions must not overlap) with
 *   16-byte loads and non-temporal stores. It calibrates the achievable HBM
 *   rate that the streaming M / M^T kernel is compared with. hip_stream: a
 *   hipStream_t or NULL. Asynchronous.
 */
int ufg_device_copy(const void* src, void* dst, long long bytes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* UFG_H */

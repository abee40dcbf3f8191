/*
 * scdyson -- lattice strong-coupling Dyson solver for MI355X (gfx950).
 *
 * Computes the lowest-order lattice Green's function of the nonequilibrium
 * strong-coupling expansion of Dirks, Mikelsons, Krishnamurthy and Freericks,
 * arXiv:1309.5994: the trapped 2D Fermi-Hubbard model of eq. (model) on the
 * discretised Kadanoff-Baym-Keldysh contour (Sec. IV.A, Fig. 1), with
 *
 *     G = S + S D G                                     (eq. Glatt, Sigma = 0)
 *
 * where S = blockdiag(S_i) holds each site's atomic-limit contour Green's
 * function (Sec. III) and D is the nearest-neighbour hopping, diagonal in
 * contour time with the quadrature weight of each contour point
 * (eq. Ginvblockstruct).  The solve is the Dyson series of App. C summed by
 * Jacobi sweeps X <- X0 + S D X over blocks of source-site columns
 * (eq. blockedGMRESproblem), each sweep one fused hopping-stencil +
 * batched complex contour GEMM on the MFMA units.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Contour: N_t = 2 n_real + n_imag points in contour order.
 *   forward   a in [0, n_real):          t = t_min + a dt,              weight +dt
 *   backward  a in [n_real, 2 n_real):   t = t_min + (2 n_real-1-a) dt, weight -dt
 *   imaginary a = 2 n_real + m:          z = t_min - i (m+1) dtau,      weight -i dtau,
 *             dtau = beta / n_imag.
 *   The same-time partner (t + 0^+) of forward point a is 2 n_real - 1 - a.
 * Lattice: Lx x Ly sites, site i = x * Ly + y, nearest neighbours
 *   (x-1,y), (x+1,y), (x,y-1), (x,y+1) in that slot order; open edges drop the
 *   bond, periodic lattices (periodic != 0) need Lx, Ly >= 3.
 * Complex numbers are interleaved (re, im) doubles (C99 double complex).
 * Inputs given per forward time (U, J) hold n_real values; the backward branch
 * uses the value at the same physical time, the imaginary branch the value at
 * t_min.
 * Every pointer named "device" must be device memory of the current HIP
 * device; "host" pointers are read before the call returns.  The caller owns
 * all memory; the library allocates nothing and keeps no pointer after a call
 * returns.  Arguments are validated before any work is enqueued.  Calls are
 * re-entrant given distinct output and workspace buffers.  `stream` is a
 * hipStream_t (NULL = the null stream).
 */
#ifndef SCDYSON_H
#define SCDYSON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define SCD_OK          0
#define SCD_EINVAL     -1   /* bad argument: null pointer, size or range        */
#define SCD_ENOMEM     -2   /* workspace smaller than scd_workspace_bytes()     */
#define SCD_EHIP       -3   /* HIP runtime error; scd_last_error() has the text */
#define SCD_ENOTCONV   -4   /* max_iter reached; outputs hold the last iterate  */
#define SCD_EDIVERGED  -5   /* sweep increments grew for 8 sweeps in a row      */
#define SCD_ENAN       -6   /* a NaN or Inf appeared in an iterate              */

/* Sweep precision for dyson_iterate. */
#define SCD_PREC_FP64   0   /* complex128 sweeps on FP64 MFMA                   */
#define SCD_PREC_FP32   1   /* complex64 FP32-MFMA correction sweeps + FP64 refinement */
#define SCD_PREC_BF16X3 2   /* complex64 correction sweeps on BF16 MFMA with split
                               products (x = hi + lo in bf16; a b ~ a_hi b_hi +
                               a_hi b_lo + a_lo b_hi, FP32 accumulation; Henry, Tang
                               & Heinecke, ARITH 2019) + FP64 refinement        */

typedef struct scd_problem {
    int32_t Lx, Ly;      /* lattice extent                                      */
    int32_t periodic;    /* 0 = open, 1 = periodic in both directions           */
    int32_t n_real;      /* forward (= backward) real-time points, >= 1         */
    int32_t n_imag;      /* imaginary-branch points, >= 1                       */
    double  dt;          /* real-time step, > 0                                 */
    double  beta;        /* inverse temperature of the initial state, > 0       */
    double  mu;          /* chemical potential                                  */
    double  t_min;       /* first real time, where the imaginary branch attaches */
} scd_problem;

typedef struct scd_stats {
    int32_t status;         /* return code of the call                          */
    int32_t n_blocks;       /* column blocks processed                          */
    int32_t sweeps_total;   /* sweeps summed over blocks (all precisions)       */
    int32_t sweeps_max;     /* largest sweep count of one block                 */
    int32_t fp64_sweeps;    /* of which FP64 sweeps                             */
    int32_t lowp_sweeps;    /* of which low-precision correction sweeps         */
    double  final_err;      /* largest final relative increment (or residual) over blocks */
    double  rho_est;        /* largest final contraction-ratio estimate e_n / e_{n-1}     */
    double  gemm_flops;     /* algorithmic contour-GEMM flops: 8 N_t^3 per (target, source)
                               pair inside the sweep's light cone (8 flops per complex MAC) */
    double  seconds;        /* host wall time of the call                       */
    double  sweep_kernel_seconds; /* summed HIP-event time of the FP64 sweep kernels */
    double  lowp_kernel_seconds;  /* summed HIP-event time of the FP32 correction sweeps */
    int32_t sweep_launches; /* FP64 sweep-kernel launches timed                 */
    int32_t lowp_launches;  /* FP32 correction-sweep launches timed             */
    double  stream_kernel_seconds; /* dyson_gmres: summed HIP-event time of the
                               streaming kernels (Gram-Schmidt passes, Givens
                               rotations, solution update)                      */
    double  stream_bytes;   /* dyson_gmres: algorithmic HBM bytes those kernels move
                               (every Krylov vector read or written once per pass) */
    int32_t stream_launches;/* dyson_gmres: streaming-kernel launches timed     */
    int32_t reserved;       /* zero                                             */
} scd_stats;

/*
 * Device workspace (bytes) that dyson_iterate needs for n_src source sites
 * processed in column blocks of block_sites sources at precision prec.
 * Returns SCD_OK and writes *bytes, or SCD_EINVAL.
 */
int scd_workspace_bytes(const scd_problem* p, int32_t n_src, int32_t block_sites,
                        int32_t prec, size_t* bytes);

/*
 * Atomic-limit contour Green's function of every site (Sec. III; the
 * number-basis evaluation with the tabulated phases of eq. cumulanttabulation).
 *   S_i[a][b] = -i [p0 e^{-i(th1_a - th1_b)} + p1 e^{-i(th2_a - th2_b)}]   a > b
 *             = +i [p2 e^{-i(th1_a - th1_b)} + p3 e^{-i(th2_a - th2_b)}]   a <= b
 * with eps_i = V_i - U(t_min)/2 - mu (eq. onsitelevels), p_nu the Boltzmann
 * weights of the four number states at t_min (energies 0, eps, eps, 2 eps + U),
 * th1 = int eps dz and th2 = int (eps + U(z)) dz along the contour from t_min
 * (trapezoid rule for U on the forward grid).
 *   V  device double[Lx*Ly]          trap potential per site
 *   U  device double[n_real]         interaction per forward time
 *   S  device complex128[N_r][N_t][N_t] output, row a contiguous
 * Errors: SCD_EINVAL (bad sizes / nulls), SCD_EHIP.
 */
int sigma_build(const scd_problem* p, const double* V, const double* U, void* S,
                void* stream);

/*
 * Solve G = S + S D G for the columns of the listed source sites.
 *   S          device complex128[N_r][N_t][N_t] from sigma_build
 *   J          device double[n_real]       hopping per forward time (all bonds)
 *   src        host int32[n_src]           source sites, each in [0, N_r)
 *   block_sites sources per column block (1..n_src); the block's iterate is
 *              N_r x N_t x block_sites*N_t complex, sized for HBM by the caller
 *   prec       SCD_PREC_FP64, SCD_PREC_FP32 or SCD_PREC_BF16X3
 *   tol        stop when the relative max-norm increment of a sweep (FP64) or
 *              the relative FP64 residual (FP32 / BF16x3 + refinement) falls below tol,
 *              with the contraction-corrected estimate e_n rho/(1-rho) also below tol
 *   max_iter   sweep limit per block (FP64 sweeps for the refined precisions)
 *   G_cols     device complex128[N_r][N_t][n_src*N_t] or NULL: full columns,
 *              column (s, b) = source src[s], contour time b
 *   G_loc      device complex128[n_src][N_t][N_t]: G(src[s], src[s]) blocks
 *   G_nn       device complex128[n_src][4][N_t][N_t]: G(nbr_d(src[s]), src[s]),
 *              zero where the neighbour slot is empty
 *   ws         device workspace of at least scd_workspace_bytes() bytes
 *   st         host stats (may be NULL)
 * Blocks the calling thread until every block has converged (one small
 * device-to-host copy per sweep).  On SCD_ENOTCONV / SCD_EDIVERGED / SCD_ENAN
 * the outputs of the failing block hold its last iterate and st is filled.
 */
int dyson_iterate(const scd_problem* p, const void* S, const double* J,
                  const int32_t* src, int32_t n_src, int32_t block_sites,
                  int32_t prec, double tol, int32_t max_iter,
                  void* G_cols, void* G_loc, void* G_nn,
                  void* ws, size_t ws_bytes, scd_stats* st, void* stream);

/*
 * Device workspace (bytes) that dyson_iterate_sym needs for the sources src
 * (host int32[n_src]) in column blocks of block_sites representatives.
 */
int scd_sym_workspace_bytes(const scd_problem* p, const int32_t* src, int32_t n_src,
                            int32_t block_sites, int32_t prec, size_t* bytes);

/*
 * dyson_iterate reduced by the lattice's point group (App. A).  When every
 * site's atomic Green's function is invariant under the point group about the
 * lattice centre (C4v for Lx == Ly: the two mirrors and the diagonal; C2v for
 * Lx != Ly), so is G: G(g(i), g(j)) = G(i, j) for every element g (the
 * hopping is uniform).  Only one source per orbit is solved (the smallest
 * site index of each orbit the requested sources meet: 36 of 256 on a 16x16
 * lattice), and the outputs of every requested source s = g(r) are copied from
 * its representative r, target sites mapped by g^-1 and neighbour slots
 * relabelled; they are bitwise those of r.
 * Arguments, outputs and errors as dyson_iterate (block_sites counts
 * representatives; the workspace is scd_sym_workspace_bytes()), plus
 * SCD_EINVAL if max |S_i - S_g(i)| over the group's generators exceeds 1e-12
 * (checked on the device before any sweep).
 */
int dyson_iterate_sym(const scd_problem* p, const void* S, const double* J,
                      const int32_t* src, int32_t n_src, int32_t block_sites,
                      int32_t prec, double tol, int32_t max_iter,
                      void* G_cols, void* G_loc, void* G_nn,
                      void* ws, size_t ws_bytes, scd_stats* st, void* stream);

/*
 * dyson_iterate (FP64) with the far blocks truncated: the columns of source j
 * are solved on the sites within lattice distance max_radius of j only (the
 * Dyson equation restricted to those sites; G is zero beyond).  G decays with
 * the distance from the source (about a decade per two hops on the 16x16
 * trap), so a radius whose outer blocks lie below the accuracy wanted
 * (App. C: only blocks in the spatial vicinity of the source matter) saves
 * the sweeps' work on the far (target, source) pairs.  max_radius >= the
 * lattice diameter reproduces dyson_iterate exactly.  Workspace as
 * scd_workspace_bytes(..., SCD_PREC_FP64); other arguments and errors as
 * dyson_iterate.
 */
int dyson_iterate_trunc(const scd_problem* p, const void* S, const double* J,
                        const int32_t* src, int32_t n_src, int32_t block_sites,
                        int32_t max_radius, double tol, int32_t max_iter,
                        void* G_cols, void* G_loc, void* G_nn,
                        void* ws, size_t ws_bytes, scd_stats* st, void* stream);

/*
 * Device workspace (bytes) that dyson_gmres needs for n_src source sites in
 * column blocks of block_sites sources with `restart` Krylov vectors per cycle.
 * Returns SCD_OK and writes *bytes, or SCD_EINVAL.
 */
int scd_gmres_workspace_bytes(const scd_problem* p, int32_t n_src, int32_t block_sites,
                              int32_t restart, size_t* bytes);

/*
 * Solve G = S + S D G for the columns of the listed source sites by
 * preconditioned restarted GMRES (App. C), the solver the paper uses.  Every
 * column (s, b) of a block is the unit-vector system A x = e of
 * eq. blockedGMRESproblem with A = B - J (eq. Ginvblockstruct) and the
 * block-diagonal preconditioner P = B^-1 = S (eq. definitionB, lowest order):
 *     (I - S D) u = S e,   start u0 = S e,
 * and GMRES(restart) minimises each column's preconditioned residual
 * |S e - (I - S D) u|_2 over u0 + K_d(I - S D, z0).  All columns of a block
 * advance in lock step: one batched matvec per Arnoldi step (the fused
 * stencil + contour GEMM of the sweeps), then per-column Gram-Schmidt
 * (classical, applied twice), Hessenberg column and Givens rotation.  It
 * converges also where the Dyson series diverges (spectral radius of S D >= 1).
 *   restart    Krylov vectors per cycle, 1..16; the workspace holds restart + 2
 *              iterates of a block (size block_sites to fit HBM)
 *   tol        stop when every column's preconditioned residual 2-norm is at most
 *              tol times the 2-norm of its S e: a cycle ends early when the
 *              rotated Hessenberg system says so (checked after every Arnoldi
 *              step), and the residual recomputed in FP64 from the iterate decides
 *   max_iter   Arnoldi steps (batched matvecs) per block
 *   other arguments as dyson_iterate; FP64 throughout.
 * st: sweeps_total / sweeps_max count Arnoldi steps; fp64_sweeps every batched
 * matvec including the residual recomputed at each (re)start; final_err the
 * largest relative residual; rho_est the mean residual reduction per step.
 * Errors as dyson_iterate (GMRES residuals never grow, so no SCD_EDIVERGED).
 */
int dyson_gmres(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                int32_t n_src, int32_t block_sites, int32_t restart, double tol,
                int32_t max_iter, void* G_cols, void* G_loc, void* G_nn, void* ws,
                size_t ws_bytes, scd_stats* st, void* stream);

/*
 * Local observables of Sec. III.A from the blocks dyson_iterate returns.
 *   n_s(t_a)     = Im G_loc[s][a][b(a)]                    (occupancy per spin)
 *   ekin_s(t_a)  = Re(-i sum_d J(t_a) G_nn[s][d][a][b(a)] ) (kinetic energy per spin:
 *                  the expectation of the site's hopping terms; G is the propagator of
 *                  hopping +J, the gauge image of eq. model's -J, so Sec. III.A's
 *                  +i sum J G with the Hamiltonian's amplitude reads -i sum J G here)
 * for forward points a in [0, n_real), b(a) = 2 n_real - 1 - a.
 *   G_loc  device complex128[n_src][N_t][N_t]
 *   G_nn   device complex128[n_src][4][N_t][N_t] (may be NULL if ekin_out is NULL)
 *   J      device double[n_real]
 *   n_out  device double[n_src][n_real]
 *   ekin_out device double[n_src][n_real] or NULL
 */
int local_observables(const scd_problem* p, const void* G_loc, const void* G_nn,
                      const double* J, int32_t n_src, double* n_out, double* ekin_out,
                      void* stream);

/*
 * Double occupancy D_s(t_a) = <n_up n_down> of each source site (Sec. III.A,
 * eq. docc), from the blocks dyson_iterate returns:
 *     U(t_a) D = Re dG - eps_j n_s(t_a) - ekin_s(t_a),   j = src[s],
 * with dG the time derivative of G_loc at equal times taken one-sided as in
 * App. B, t' = t^+ held at the backward point b(a) of the same time:
 * (G_loc[s][a][b(a)] - G_loc[s][a-1][b(a)]) / dt for a >= 1 and
 * (G_loc[s][1][b(0)] - G_loc[s][0][b(0)]) / dt at a = 0, and
 * eps_j = V_j - U(t_min)/2 - mu.  Discretisation error O(dt) (O(dt^2) for
 * constant U); combine runs at several dt with scd_extrapolate_dt.
 *   G_loc, G_nn  device, as local_observables (G_nn required)
 *   J, U         device double[n_real];  V device double[N_r]
 *   src          DEVICE int32[n_src]: the site of each block
 *   d_out        device double[n_src][n_real]
 *   frac_out     device double[n_real] or NULL: the doubly occupied fraction
 *                2 sum_s D_s / (2 sum_s n_s) of the listed sites (Sec. V.B)
 * Needs n_real >= 2; D is Inf/NaN where U(t_a) = 0.
 */
int double_occupancy(const scd_problem* p, const void* G_loc, const void* G_nn,
                     const double* J, const double* V, const double* U,
                     const int32_t* src, int32_t n_src, double* d_out, double* frac_out,
                     void* stream);

/*
 * dt -> 0 extrapolation of results at two or three step sizes (Sec. IV.D:
 * linear or quadratic in dt): out[i] = value at dt = 0 of the polynomial
 * through (dts[k], values[k][i]).  Host memory; values sampled at the same
 * physical times for every dt.  SCD_EINVAL for n_dt not 2 or 3 or equal
 * step sizes.
 */
int scd_extrapolate_dt(const double* dts, int32_t n_dt, const double* values, int32_t n,
                       double* out);

/*
 * Device workspace (bytes) of sigma2_build and sigma2_dress.
 */
int scd_sigma2_workspace_bytes(const scd_problem* p, size_t* bytes);

/*
 * Second-order strong-coupling self-energy of every site (Sec. III,
 * eq. defnSigmatilde), paramagnetic:
 *   Sigma~_i(a, b) = - sum_{s1 = up, dn} sum_{c, d} G~_{up s1}(a, d; c, b) K_i(c, d),
 *   K_i(c, d) = w_c J(z_c) [sum_{k in nbr(i)} G_loc,k(c, d)] J(z_d) w_d,
 * with the cumulant G~_{s s1}(t1, t2; t1', t2') = G^II + G(t1,t1') G(t2,t2') delta_{s s1}
 * - G(t1,t2') G(t2,t1') of the on-site two-particle propagator
 * G^II = (-i)^2 <T_C c_s(t1) c_s1(t2) c^dag_s1(t1') c^dag_s(t2')>, evaluated on the fly in
 * the number basis from the tabulated phases (eq. cumulanttabulation) and the
 * Boltzmann weights at t_min; G = S_i.  At equal contour indices creation operators
 * count as later than annihilation operators.
 *   V, U, J     device double[N_r], [n_real], [n_real] (as sigma_build / dyson_iterate)
 *   S           device complex128[N_r][N_t][N_t] from sigma_build
 *   G_loc_all   device complex128[N_r][N_t][N_t]: the local Green's function of every
 *               site in site order (dyson_iterate with src = 0..N_r-1)
 *   sig_out     device complex128[N_r][N_t][N_t]
 *   ws          device workspace of scd_sigma2_workspace_bytes()
 * Cost: O(N_r N_t^4) on the vector units.
 */
int sigma2_build(const scd_problem* p, const double* V, const double* U, const double* J,
                 const void* S, const void* G_loc_all, void* sig_out, void* ws,
                 size_t ws_bytes, void* stream);

/*
 * Dressed block diagonal for eq. Glatt with the self-energy Sigma =
 * calG^-1 o Sigma~ o calG^-1 (eq. defnSigma; contour products carry the
 * quadrature weights): the contour inverse of calG_i^-1 - Sigma_i is
 *   S'_i = S_i (S_i - Sigma~_i)^-1 S_i,
 * so dyson_iterate with S' in place of S solves the lattice Dyson equation with
 * Sigma.  Gauss-Jordan elimination with partial pivoting per site.
 *   S, sig   device complex128[N_r][N_t][N_t];  S_out the same (not aliasing S)
 * Errors: SCD_ENAN if S - Sigma~ is singular on a site.  Blocks until done.
 */
int sigma2_dress(const scd_problem* p, const void* S, const void* sig, void* S_out, void* ws,
                 size_t ws_bytes, void* stream);

/*
 * Device workspace (bytes) of dyson_selfconsistent.
 */
int scd_selfconsistent_workspace_bytes(const scd_problem* p, int32_t block_sites, int32_t prec,
                                       size_t* bytes);

/*
 * The self-consistent second-order strong-coupling solution (Sec. III):
 * S = sigma_build(V, U); Sigma~ = 0; repeat
 *     G_loc of every site = dyson_iterate with the dressed blocks sigma2_dress(S, Sigma~),
 *     Sigma~_new = sigma2_build(G_loc),
 *     d = |Sigma~_new - Sigma~|_F / N_bd + max |Sigma~_new - Sigma~|,  N_bd = N_r N_t^2,
 *     Sigma~ = lam Sigma~_new + (1 - lam) Sigma~                   (eq. Sigmamix)
 * until d <= delta_sc, then one last solve with the final Sigma~ (the norm is
 * taken on Sigma~, of which Sigma = calG^-1 o Sigma~ o calG^-1 is a fixed
 * linear image; the paper uses lam ~ 0.7 and delta_sc ~ 1e-8 U).
 *   V, U, J      device inputs as sigma_build / dyson_iterate
 *   lam          mixing parameter in (0, 1];  delta_sc > 0;  max_sc >= 1 steps
 *   block_sites, prec, tol, max_iter   passed to every dyson_iterate (all N_r sources)
 *   S_out        device complex128[N_r][N_t][N_t]: the atomic S
 *   sig_out      device complex128[N_r][N_t][N_t]: the final Sigma~
 *   G_loc, G_nn  device complex128[N_r][N_t][N_t], [N_r][4][N_t][N_t] (G_nn may be NULL)
 *                of the last solve, in site order
 *   sc_iter, sc_norm  host (nullable): steps taken and the last d
 *   st           host (nullable): the lattice solves' statistics summed
 * Errors as dyson_iterate and sigma2_dress; SCD_ENOTCONV if d > delta_sc after
 * max_sc steps (outputs hold the last state).  Blocks until done.
 */
int dyson_selfconsistent(const scd_problem* p, const double* V, const double* U, const double* J,
                         double lam, double delta_sc, int32_t max_sc, int32_t block_sites,
                         int32_t prec, double tol, int32_t max_iter, void* S_out, void* sig_out,
                         void* G_loc, void* G_nn, void* ws, size_t ws_bytes, int32_t* sc_iter,
                         double* sc_norm, scd_stats* st, void* stream);

/*
 * Device workspace (bytes) for dyson_adjoint at precision prec.
 */
int scd_adjoint_workspace_bytes(const scd_problem* p, int32_t prec, size_t* bytes);

/*
 * Densities at one forward time and the adjoint of a weighted density loss
 *     L = sum_l w_l n_l(t_e),   n_l(t_e) = Im G[(l, e), (l, b(e))]   (Sec. III.A)
 * for the Dyson solve G = S + S D G.  With G = (I - S D)^-1 S one needs, per
 * site l, the forward column g_l = G v_l (v_l: unit vector at (l, b(e))) and
 * the transposed-system column h_l = G^T u_l = (I - S^T D)^-1 S^T u_l
 * (u_l: unit vector at (l, e)); both are solved by the same sweep kernels
 * with one column per site (the forward columns are recomputed, nothing is
 * stored between calls).  Then
 *     dL/dS_j = sum_l w_l (u_l + D h_l)_j (v_l + D g_l)_j^T,
 *     dL/dJ(z_c) = Im w_c sum_l w_l sum_i h_l[(i,c)] sum_{k in nbr(i)} g_l[(k,c)],
 * chained through the closed form of S (eps_j = V_j - U(t_min)/2 - mu, the
 * Boltzmann weights and the phase integral of U).  Gradients with respect to
 * J(t) and U(t) sum every contour point that carries the physical time t.
 *   S        device complex128[N_r][N_t][N_t] from sigma_build
 *   V, U     device double[N_r], double[n_real] (inputs of sigma_build; needed for gradients)
 *   J        device double[n_real]
 *   w_loss   device double[N_r] loss weights (needed for loss or gradients)
 *   t_index  forward time index e in [0, n_real)
 *   prec, tol, max_iter   as for dyson_iterate (applied to both solves)
 *   n_te     device double[N_r] or NULL: n_l(t_e) for every site
 *   loss     device double[1] or NULL: L
 *   dV, dU, dJ  device double[N_r], [n_real], [n_real]: all three, or all NULL
 *              (then only the forward columns are solved)
 *   ws       device workspace of scd_adjoint_workspace_bytes() bytes
 * Errors as dyson_iterate.
 */
int dyson_adjoint(const scd_problem* p, const void* S, const double* V, const double* U,
                  const double* J, const double* w_loss, int32_t t_index, int32_t prec,
                  double tol, int32_t max_iter, double* n_te, double* loss, double* dV,
                  double* dU, double* dJ, void* ws, size_t ws_bytes, scd_stats* st,
                  void* stream);

/* Message for the last failing call on this thread ("" if none). */
const char* scd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SCDYSON_H */

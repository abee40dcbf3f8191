// Internal declarations shared by the scdyson translation units (not installed).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <vector>

#include "scdyson.h"

namespace scd {

// Largest contour length the sweep kernels are instantiated for (row tiles of
// 16 contour points, 1..kMaxRowTiles).
constexpr int kTile = 16;
constexpr int kMaxRowTiles = 16;
constexpr int kMaxNt = kTile * kMaxRowTiles;     // 256
constexpr int kColsPerWG = 32;                   // column tile of one sweep workgroup

typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef double dvec4 __attribute__((ext_vector_type(4)));
typedef float fvec4 __attribute__((ext_vector_type(4)));

// Geometry of one problem, derived on the host from scd_problem.
struct Geom {
    int Lx, Ly, periodic;
    int n_r;        // sites
    int n_real, n_imag;
    int n_t;        // contour points
    int mt;         // row tiles: n_t padded to mp = 16 * mt
    int mp;
    double dt, beta, mu, t_min, dtau;
};

// Parameters of one sweep launch (one column block).
struct SweepArgs {
    int Lx, Ly, periodic;
    int n_r, n_t;
    int ldx;        // padded column count of the block iterate (multiple of kColsPerWG)
    int ntn;        // column tiles per site = ldx / kColsPerWG
    int bs;         // source sites in this block
    int lc_sweep;   // sweeps already applied (light cone radius) or -1 to disable skipping
    int group;      // tile order: groups of `group` consecutive sites, column tile major inside
    int x0_kind;    // X0_BLOCK, X0_COL or X0_COL_T (what X0 holds on a source's own site)
    int x0_fixed;   // the fixed contour index of X0_COL / X0_COL_T
    const int* sites;  // sites updated by this launch (one colour of a red-black
                       // sweep), or nullptr for all sites in index order
    int n_sites;    // number of updated sites
    int part_off;   // offset (in workgroups) of this launch's convergence partials
    int check;      // 1: read old values and reduce the increment; 0: write only
    void* out2 = nullptr;  // RESIDUAL: second destination of R (the start of the
                           // correction sweeps), or nullptr
    int no_x0 = 0;         // SOLVE: leave out X0, Y = St^T N(X) (the batched matvec of GMRES)
    int out_f64 = 0;       // RESIDUAL: write R as complex128 instead of complex64
    int max_radius = -1;   // SOLVE: truncation radius (lattice distance from a column's
                           // source beyond which G is zero), or -1
};

// X0 of a column block (the preconditioned unit-vector bundle):
//  X0_BLOCK  column (s, b) = S_j[:, b] on site j = src[s] (all N_t columns per source)
//  X0_COL    column s      = S_j[:, fixed]  (one column per source)
//  X0_COL_T  column s      = S_j[fixed, :]  (one column per source, transposed system)
enum { X0_BLOCK = 0, X0_COL = 1, X0_COL_T = 2 };

// Logical tile -> (site, column tile).  Sites are taken in groups of `group`
// consecutive sites; inside a group the column tile is the slow index, so the
// workgroups that run together share neighbour tiles of the iterate.
__host__ __device__ inline void tile_site_col(int tile, int ntn, int n_r, int group, int* site,
                                              int* ct) {
    const int g = tile / (group * ntn);
    const int first = g * group;
    const int cnt = (n_r - first) < group ? (n_r - first) : group;
    const int local = tile - first * ntn;
    *ct = local / cnt;
    *site = first + (local - (local / cnt) * cnt);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Site neighbours in slot order (x-1,y), (x+1,y), (x,y-1), (x,y+1); -1 if absent.
__host__ __device__ inline void site_neighbours(int i, int Lx, int Ly, int periodic, int nb[4]) {
    const int x = i / Ly, y = i - (i / Ly) * Ly;
    int xs[4] = {x - 1, x + 1, x, x};
    int ys[4] = {y, y, y - 1, y + 1};
    for (int d = 0; d < 4; ++d) {
        int xx = xs[d], yy = ys[d];
        if (periodic) {
            xx = (xx + Lx) % Lx;
            yy = (yy + Ly) % Ly;
            nb[d] = xx * Ly + yy;
        } else {
            nb[d] = (xx >= 0 && xx < Lx && yy >= 0 && yy < Ly) ? xx * Ly + yy : -1;
        }
    }
}

// Hopping weight w(z_c) * J(z_c) of contour point c, as (re, im).
__device__ inline double2 contour_wj(int c, int n_real, double dt, double dtau, const double* J) {
    if (c < n_real) return make_double2(dt * J[c], 0.0);
    if (c < 2 * n_real) return make_double2(-dt * J[2 * n_real - 1 - c], 0.0);
    return make_double2(0.0, -dtau * J[0]);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tiles so tiles sharing operands share an L2.
__device__ inline int xcd_remap(int bid, int nb) {
    const int per = nb >> 3;
    if (bid >= (per << 3)) return bid;
    return (bid & 7) * per + (bid >> 3);
}

// ---- tile order (order.hip) ----
// Sites per tile-order group (SCD_SITE_GROUP overrides the default).
int site_group(const Geom& g);
// Square lattice patches of the colour order (SCD_PATCH overrides).
int colour_patch(const Geom& g);
// Launch site list: the two colours of a bipartite lattice (*n_even = size of
// the first) or all sites, each interleaved over the XCDs in groups.
std::vector<int32_t> colour_order(const Geom& g, int group, bool bipartite, int* n_even);

// ---- launchers (each returns hipError_t of the launch) ----
hipError_t launch_sigma_build(const Geom& g, const double* V, const double* U, double2* S,
                              hipStream_t st);
hipError_t launch_scale_transpose(const Geom& g, const double2* S, const double* J, double2* St,
                                  int transposed_system, hipStream_t st);
hipError_t launch_init_block(const Geom& g, const double2* S, const int* src_blk, int bs, int ldx,
                             int x0_kind, int x0_fixed, double2* X, double2* Xn, hipStream_t st);
hipError_t launch_sweep_f64(const Geom& g, const SweepArgs& a, const double2* St, const double2* S,
                            const int* src_blk, const double2* X, double2* Xn, double* partial,
                            hipStream_t st);
hipError_t launch_residual_f64(const Geom& g, const SweepArgs& a, const double2* St,
                               const double2* S, const int* src_blk, const double2* X, void* R32,
                               double* partial, hipStream_t st);
hipError_t launch_correct_f32(const Geom& g, const SweepArgs& a, const void* St32,
                              const int* src_blk, const void* R32, const void* D32, void* Dn32,
                              double* partial, hipStream_t st);
hipError_t launch_to_f32(const double2* in, void* out, size_t n, hipStream_t st);
// BF16x3 correction sweep (sweep_bf3.hip): operand bytes for g, operand build
// from St (complex128 [n_r][mp][mp]), and the sweep D' = R + St^T N(D) with
// one convergence partial per workgroup, as the other sweep launchers.
size_t bf3_operand_bytes(const Geom& g);
hipError_t launch_bf3_operand(const Geom& g, const double2* St, void* out, hipStream_t st);
hipError_t launch_correct_bf3(const Geom& g, const SweepArgs& a, const void* Abf,
                              const int* src_blk, const void* R32, const void* D32, void* Dn32,
                              double* partial, hipStream_t st);
// ---- second-order self-energy (sigma2.hip) ----
hipError_t launch_sigma2(const Geom& g, const double* V, const double* U, const double* J,
                         const double2* S, const double2* G_loc_all, double2* K, double2* part,
                         double2* M, double2* sig, hipStream_t st);
hipError_t launch_dress(const Geom& g, const double2* S, const double2* sig, double2* aug,
                        double2* S_out, int* singular, hipStream_t st);
// sig <- lam fresh + (1 - lam) sig; part[2 w] = sum |fresh - sig|^2, part[2 w + 1] =
// max |fresh - sig| over the elements of workgroup w (n_part workgroups).
hipError_t launch_mix(const double2* fresh, double2* sig, double lam, size_t n, double* part,
                      int n_part, hipStream_t st);

// ---- point-group reduction (sym.hip) ----
// The lattice's point group about its centre: C4v (8 elements) for Lx == Ly,
// else C2v (4).  Element e applies mirror x (bit 0), mirror y (bit 1), then
// the diagonal swap (bit 2).
struct SymGroup {
    int n_el = 0;
    std::vector<int> perm, perm_inv;   // [n_el][n_r]: site images under e and e^-1
    std::vector<int> rep, elem;        // per site: orbit representative (smallest
                                       // index) and an element taking it to the site
};
SymGroup lattice_group(const Geom& g);
// Neighbour slot of rep(s) that slot d of s maps to under elem(s)^-1 (-1: no
// neighbour; -2: the element does not preserve the neighbour structure).
int sym_slot(const SymGroup& G, const Geom& g, int s, int d);
hipError_t launch_sym_check(const double2* S, const int* perm, const Geom& g, double* part,
                            int n_part, hipStream_t st);
hipError_t launch_extract_sym(const Geom& g, const double2* X, int ldx, const int* src_blk,
                              const int* req, const int* req_lr, const int* req_g,
                              const int* req_slot, const int* perm_inv, int n_req, int n_src,
                              double2* G_cols, double2* G_loc, double2* G_nn, hipStream_t st);

// ---- batched GMRES (gmres.hip) ----
// Krylov vectors a cycle may dot against (the restart length limit).
constexpr int kMaxBasis = 16;
enum { GS_DOTS = 0, GS_PROJ_DOTS = 1, GS_UPDATE_NORM = 2, GS_NORM = 3, GS_UPDATE = 4 };
// One streaming pass over the basis q_i = sig_i v_i (i < k) and a vector w.
struct GsPass {
    const double2* Q;     // v_0; v_i at Q + i * qstride
    size_t qstride;       // elements between basis vectors
    int k;                // basis vectors used
    const double* sig;    // [kMaxBasis + 1][ldx] column scales of the basis
    double2* w;           // vector read (and written by the UPDATE passes)
    const double* wsig;   // [ldx] column scale applied to w on reading, or nullptr
    const double2* coef;  // UPDATE: c_i = sum over parts of coef[part][i][column]
    const double2* coef2; //   (+ the same sum over coef2 if not nullptr)
    int coef_parts;
    size_t coef_pstride;  // elements between parts
    double2* pdot;        // DOTS: [chunk][kMaxBasis][ldx] partial <q_i, x>
    double* pnorm;        // NORM: [chunk][ldx] partial |x|^2
    int rows, ldx, chunk_rows;   // chunk_rows: a multiple of mp (whole sites)
    // Light cone: every vector of the pass vanishes on sites farther than
    // `radius` from the source of a column; a workgroup whose sites and
    // sources are all farther apart skips its rows (radius < 0: no skipping).
    const int* src_blk;
    int radius, bs, n_t, mp, Lx, Ly, periodic;
};
// Per-column Hessenberg / Givens state of one Arnoldi step d (d < 0: cycle start).
struct GivensArgs {
    const double2* pa;    // [nch][kMaxBasis][ldx] first Gram-Schmidt dots
    const double2* pb;    // [nch][kMaxBasis][ldx] second Gram-Schmidt dots
    const double* pn;     // [nch][ldx] partial squared norms
    int nch, d, ldx;
    double* sig;          // [kMaxBasis + 1][ldx]: writes sig[d + 1] (sig[0] at a start)
    double2* R;           // [kMaxBasis][kMaxBasis][ldx] rotated Hessenberg (row, column)
    double* cs;           // [kMaxBasis][ldx] rotation cosines
    double2* sn;          // [kMaxBasis][ldx] rotation sines
    double2* gv;          // [kMaxBasis + 1][ldx] rotated right-hand side
    const double* x0n;    // [ldx] |S e| of every column
    double* part;         // per-workgroup (max residual ratio, 1, bad) triples
};
int gs_chunks(int rows, int ldx);
hipError_t launch_gs(int mode, const GsPass& p, hipStream_t st);
hipError_t launch_givens(const GivensArgs& a, hipStream_t st);
hipError_t launch_gmres_solve(const double2* R, const double2* gv, double2* y, int k, int ldx,
                              hipStream_t st);
hipError_t launch_colnorm(const double* pn, int nch, int ldx, double* out, hipStream_t st);

hipError_t launch_axpy_f32_to_f64(double2* X, const void* D32, size_t n, hipStream_t st);
hipError_t launch_adjoint_grads(const Geom& g, int ldx, int e, const double2* H, const double2* Gc,
                                const double* V, const double* U, const double* J, const double* w,
                                double2* Lam, double2* rsum, double2* csum, double* bz, double* djc,
                                double* dV, double* dU, double* dJ, hipStream_t st);
hipError_t launch_adjoint_loss(const Geom& g, int ldx, int e, const double2* Gc, const double* w,
                               double* n_te, double* loss, hipStream_t st);
hipError_t launch_reduce_max3(const double* partial, int n, unsigned long long* slot,
                              hipStream_t st);
hipError_t launch_extract(const Geom& g, const double2* X, int ldx, const int* src_blk, int bs,
                          int blk_start, int n_src, double2* G_cols, double2* G_loc, double2* G_nn,
                          hipStream_t st);
hipError_t launch_docc(const Geom& g, const double2* G_loc, const double2* G_nn, const double* J,
                       const double* V, const double* U, const int* src, int n_src, double* d_out,
                       double* frac_out, hipStream_t st);
hipError_t launch_observables(const Geom& g, const double2* G_loc, const double2* G_nn,
                              const double* J, int n_src, double* n_out, double* ekin_out,
                              hipStream_t st);

}  // namespace scd

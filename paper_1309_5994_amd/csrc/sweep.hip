// One Dyson sweep of a column block, fused with its convergence measure:
//
//     Y_i = X0_i + St_i^T * sum_{k in nbr(i)} X_k
//
// the Dyson-series step of App. C of arXiv:1309.5994 applied to a bundle of
// unit vectors (eq. blockedGMRESproblem).  St_i = (S_i diag(w J))^T is the
// site's scaled atomic Green's function stored transposed (see aux.hip).
//
// Work decomposition (gfx950, 64-wide waves):
//  * one workgroup = one target site i and a 32-column tile of the block
//    iterate, all mp = 16*MT contour rows; 4 waves (one per SIMD): waves 0-1
//    own the upper MT/2 row tiles, waves 2-3 the lower MT/2, each wave one
//    16-column slice; for odd MT the last row tile is split over the k-steps
//    between the two groups, so every SIMD issues the same MFMA count.  At
//    about 200 VGPRs per wave two workgroups share a CU, and one's barriers
//    and staging overlap the other's MFMAs.
//  * K loop over contour time c in chunks of KC: the chunk of St_i
//    (contiguous KC x mp complex) and the sum of the (up to) four neighbour
//    tiles X_k[c-chunk][32 cols] are staged through double-buffered LDS (one
//    barrier per chunk); the neighbour sum is the hopping stencil, done while
//    staging so the summed tile never reaches HBM.  Global loads of chunk k+1
//    are issued before the MFMAs of chunk k.
//  * complex products as real MFMAs per 16x16x4 block on
//    V_MFMA_F64_16X16X4_F64 (FP64) or V_MFMA_F32_16X16X4_F32 (FP32): four
//    (re += ar br - ai bi, im += ar bi + ai br), or three (P1 = ar br,
//    P2 = ai bi, P3 = (ar + ai)(br + bi); re = P1 - P2, im = P3 - P1 - P2)
//    where the third accumulator fits in registers.  Flops are
//    counted as 8 per complex multiply-add either way.
//  * light cone: after n sweeps the iterate of source j is zero beyond
//    Manhattan distance n from j (the support argument of Sec. IV.D); a tile
//    whose sources are all farther than n+1 from site i is skipped (its output
//    stays zero).
//
// Red-black ordering: on a bipartite lattice the neighbours of one colour are
// all of the other colour, so a launch over one colour can update X in place
// (each workgroup reads its own tile before overwriting it and only
// neighbour tiles of the other colour); two such launches form a Gauss-Seidel
// sweep, whose contraction rate is the square of the Jacobi sweep's.
//
// Convergence checks: a launch with `check` set reads each output's old value
// and reduces max|X' - X|; other launches only write (plus max|X'| and the
// NaN/Inf flag), which saves one tile read per workgroup.  The host schedules
// checks from the measured contraction rate.
//
// Modes:
//  * SOLVE     (FP64): X0 from S (or none: the matvec St^T N(X) of GMRES);
//              writes Y; partials max|Y - X|, max|Y|.  With a truncation
//              radius, columns whose source is farther from the target stay
//              zero (the Dyson equation restricted to the sites within it).
//  * RESIDUAL  (FP64): X0 from S; writes R = Y - X as complex64 (the FP64
//              residual of iterative refinement) or complex128 (the residual
//              GMRES restarts from); partials max|R|, max|Y|.
//  * CORRECT   (FP32): X0 is a complex64 residual R; X is the correction D;
//              writes D' = R + St^T (sum of neighbours of D); partials
//              max|D' - D|, max|D'|.
// X0 kinds (SOLVE / RESIDUAL): BLOCK = whole sources, column (s, b) holds S_j[:, b]
// on site j = src[s]; COL = one column per source, S_j[:, fixed]; COL_T = one
// column per source, S_j[fixed, :] (the transposed system of the adjoint).
#include "internal.h"

namespace scd {
namespace {

constexpr int kThreads = 256;
enum { MODE_SOLVE = 0, MODE_RESIDUAL = 1, MODE_CORRECT = 2 };

struct EngF64 {
    typedef double real;
    typedef dvec2 cplx;
    typedef dvec4 acc;
    // Three real products per complex one where the third accumulator still
    // fits in 256 VGPRs without spills; in the staged-sum form (P1, P2, P3).
    static constexpr bool gauss(int mt) { return mt <= 12; }
    static constexpr bool staged_sum = true;
    __device__ static acc mma(real a, real b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // V_MFMA_F64_16X16X4_F64 result: element v of lane l is row 4 v + l/16, column l%16.
    __device__ static int row(int v, int lq) { return 4 * v + lq; }
};

struct EngF32 {
    typedef float real;
    typedef fvec2 cplx;
    typedef fvec4 acc;
    // Gauss's form (T, U, V) with its sums in the k-loop: the staged-sum form
    // costs enough registers to drop a third FP32 workgroup per CU.
    static constexpr bool gauss(int) { return true; }
    static constexpr bool staged_sum = false;
    __device__ static acc mma(real a, real b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // V_MFMA_F32_16X16X4_F32 result: element v of lane l is row 4 (l/16) + v, column l%16.
    __device__ static int row(int v, int lq) { return 4 * lq + v; }
};

// K chunk of a sweep kernel: the largest of 32, 16, 8 contour points that
// divides mp and keeps the workgroup's double-buffered LDS (St chunk,
// neighbour sum and its (br + bi) plane) within half of the CU's 160 KB, so
// two workgroups fit per CU.
template <class E>
constexpr int chunk_k(int mt) {
    typedef typename E::cplx C;
    const bool staged = E::gauss(mt) && E::staged_sum;
    const int mp = kTile * mt;
    for (int kc = 32; kc >= 8; kc /= 2) {
        // St chunk, neighbour sum and its (br + bi) plane, two buffers each
        const int bytes = kc * (2 * mp + (staged ? 3 : 2) * kColsPerWG) * (int)sizeof(C);
        if (mp % kc == 0 && bytes <= 78 * 1024) return kc;
    }
    return 8;
}

// Elements of one St staging buffer: the chunk padded to whole passes of the
// workgroup, and at least half the 8 KB through which the two row groups
// exchange the shared tile's partial sums (2 slices x 4 rows x re/im x 64
// lanes of doubles) once both buffers are free.
template <class E>
constexpr int as_stride(int mt) {
    typedef typename E::cplx C;
    const int chunk = (chunk_k<E>(mt) * kTile * mt + kThreads - 1) / kThreads * kThreads;
    const int xch = 2 * 4 * 2 * 64 * (int)sizeof(double) / 2 / (int)sizeof(C);
    return chunk > xch ? chunk : xch;
}

// Everything a wave does after the workgroup set-up.  Waves 0-1 form row
// group 0 and waves 2-3 row group 1 (GRP, a template parameter: the kernel
// picks the instantiation with one wave-uniform branch, so the MFMA stream
// carries no predicates); wave & 1 picks the 16-column slice.  Each group owns
// MT/2 row tiles; for odd MT the last tile is shared, group 0 taking the even
// and group 1 the odd k-steps of every chunk, and group 1 hands its partial
// sums to group 0 through LDS before the epilogue.  Both groups therefore
// issue the same number of MFMAs per chunk and every SIMD stays busy.
template <class E, int MT, int MODE, int GRP>
__device__ __forceinline__ void sweep_rows(const typename E::cplx* __restrict__ Sti,
                                           const typename E::cplx* const (&Xk)[4],
                                           const dvec2* __restrict__ S,
                                           const int* __restrict__ src_blk,
                                           const typename E::cplx* X, void* out,
                                           const fvec2* __restrict__ R, double* part,
                                           const SweepArgs& g, int i, int n0, int cols_per_src,
                                           typename E::cplx* As, typename E::cplx* Bs,
                                           typename E::real* Bd, double (*red)[3]) {
    typedef typename E::real real;
    typedef typename E::cplx cplx;
    typedef typename E::acc acc;
    constexpr int KC = chunk_k<E>(MT);
    constexpr int MP = kTile * MT;
    constexpr int NW = kColsPerWG;
    constexpr int NOWN = MT / 2;                      // row tiles owned by each group
    constexpr bool SHARED = (MT % 2) != 0;            // last tile split over k-steps
    constexpr int NA = NOWN + (SHARED ? 1 : 0);       // accumulator tiles per wave
    constexpr int A_ELEMS = KC * MP;
    // The St chunk goes through registers, A_PER elements per thread; each of
    // the two LDS buffers holds A_STRIDE elements (the chunk plus padding of
    // the last pass).
    constexpr int A_PER = (A_ELEMS + kThreads - 1) / kThreads;
    constexpr int A_STRIDE = as_stride<E>(MT);
    constexpr int B_ELEMS = KC * NW;
    constexpr int B_PER = B_ELEMS / kThreads;
    static_assert(MP % KC == 0, "k chunk must tile the padded contour length");
    static_assert(B_ELEMS % kThreads == 0, "B chunk must be a whole number of passes");
    static_assert((KC / 4) % 2 == 0, "the shared tile needs an even number of k-steps");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wc = wave & 1;
    const int l16 = lane & 15;
    const int lq = lane >> 4;
    const int ldx = g.ldx;
    const int t0 = GRP * NOWN;                        // first owned row tile

    // Four-product form: accr = sum ar br - ai bi, acci = sum ar bi + ai br.
    // Three-product forms (G3).  Staged-sum form (E::staged_sum): accr = P1 =
    // sum ar br, acci = P2 = sum ai bi, accg = P3 = sum (ar + ai)(br + bi);
    // re = P1 - P2, im = P3 - P1 - P2; the (br + bi) plane is staged with the
    // neighbour sum, so a k-step adds only one (ar + ai) per row tile in front
    // of its MFMAs.  Gauss's form: accr = T = sum ar (br + bi), acci = U =
    // sum (ar + ai) bi, accg = V = sum (ai - ar) br; re = T - U, im = T + V.
    constexpr bool G3 = E::gauss(MT);
    constexpr bool PS = G3 && E::staged_sum;
    acc accr[NA], acci[NA], accg[G3 ? NA : 1];
#pragma unroll
    for (int t = 0; t < NA; ++t) {
        accr[t] = acc{0, 0, 0, 0};
        acci[t] = acc{0, 0, 0, 0};
        if (G3) accg[t] = acc{0, 0, 0, 0};
    }

    cplx ra[A_PER];
    cplx rb[B_PER][4];

    // Staging of one K chunk: global -> registers, issued a chunk ahead of its
    // use, then registers -> LDS buffer `buf` (the St chunk as is, the four
    // neighbour tiles summed).  Threads past the end of the St chunk re-load
    // its last element into the buffer's padding, so no lane is predicated
    // off.
#define SCD_GLOAD(k0, buf)                                                             \
    do {                                                                               \
        _Pragma("unroll") for (int r = 0; r < A_PER; ++r) {                            \
            int e = tid + r * kThreads;                                                \
            e = e < A_ELEMS ? e : A_ELEMS - 1;                                         \
            ra[r] = Sti[(size_t)(k0) * MP + e];                                        \
        }                                                                              \
        _Pragma("unroll") for (int r = 0; r < B_PER; ++r) {                            \
            const int e = tid + r * kThreads;                                          \
            const int kk = e / NW, col = e - (e / NW) * NW;                            \
            const size_t off = (size_t)((k0) + kk) * ldx + n0 + col;                   \
            _Pragma("unroll") for (int d = 0; d < 4; ++d)                              \
                rb[r][d] = Xk[d] ? Xk[d][off] : cplx{0, 0};                            \
        }                                                                              \
    } while (0)
#define SCD_LSTORE(buf)                                                                \
    do {                                                                               \
        _Pragma("unroll") for (int r = 0; r < A_PER; ++r)                              \
            As[(buf) * A_STRIDE + tid + r * kThreads] = ra[r];                         \
        _Pragma("unroll") for (int r = 0; r < B_PER; ++r)                              \
        {                                                                              \
            const cplx v = (rb[r][0] + rb[r][1]) + (rb[r][2] + rb[r][3]);              \
            Bs[(buf) * B_ELEMS + tid + r * kThreads] = v;                              \
            if (PS) Bd[(buf) * B_ELEMS + tid + r * kThreads] = v.x + v.y;              \
        }                                                                              \
    } while (0)

    // Double-buffered LDS, one barrier per chunk: the barrier of chunk c
    // publishes its staged St chunk and neighbour sum, and proves every wave
    // done with chunk c - 1, whose buffers chunk c + 1 then overwrites.
    SCD_GLOAD(0, 0);
    for (int k0 = 0, cb = 0; k0 < MP; k0 += KC, cb ^= 1) {
        SCD_LSTORE(cb);
        __syncthreads();
        if (k0 + KC < MP) SCD_GLOAD(k0 + KC, cb ^ 1);
        const cplx* Ac = As + cb * A_STRIDE;
        const cplx* Bc = Bs + cb * B_ELEMS;
        const real* Bdc = Bd + cb * B_ELEMS;
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            // Tiles of this k-step: the owned ones, plus the shared one on
            // this group's parity.
            const bool sh = SHARED && ((s & 1) == GRP);
            const int nt = NOWN + (sh ? 1 : 0);
            const int kr = 4 * s + lq;
            const cplx b = Bc[kr * NW + wc * 16 + l16];
            cplx a[NA];
#pragma unroll
            for (int t = 0; t < NA; ++t) {
                const int tt = t < NOWN ? t0 + t : MT - 1;
                if (t < nt) a[t] = Ac[kr * MP + tt * kTile + l16];
            }
            if (PS) {
                const real bsum = Bdc[kr * NW + wc * 16 + l16];
#pragma unroll
                for (int t = 0; t < NA; ++t) {
                    if (t < nt) {
                        accr[t] = E::mma(a[t].x, b.x, accr[t]);
                        acci[t] = E::mma(a[t].y, b.y, acci[t]);
                        accg[t] = E::mma(a[t].x + a[t].y, bsum, accg[t]);
                    }
                }
            } else if (G3) {
                const real bsum = b.x + b.y;
#pragma unroll
                for (int t = 0; t < NA; ++t) {
                    if (t < nt) {
                        accr[t] = E::mma(a[t].x, bsum, accr[t]);
                        acci[t] = E::mma(a[t].x + a[t].y, b.y, acci[t]);
                        accg[t] = E::mma(a[t].y - a[t].x, b.x, accg[t]);
                    }
                }
            } else {
#pragma unroll
                for (int t = 0; t < NA; ++t) {
                    if (t < nt) {
                        accr[t] = E::mma(a[t].x, b.x, accr[t]);
                        acci[t] = E::mma(a[t].x, b.y, acci[t]);
                    }
                }
#pragma unroll
                for (int t = 0; t < NA; ++t) {
                    if (t < nt) {
                        accr[t] = E::mma(-a[t].y, b.y, accr[t]);
                        acci[t] = E::mma(a[t].y, b.x, acci[t]);
                    }
                }
            }
        }
    }
#undef SCD_GLOAD
#undef SCD_LSTORE

    // Complex partial sums of tile t, element v.
    auto part_re = [&](int t, int v) -> double {
        return G3 ? (double)accr[t][v] - (double)acci[t][v] : (double)accr[t][v];
    };
    auto part_im = [&](int t, int v) -> double {
        return PS   ? (double)accg[t][v] - (double)accr[t][v] - (double)acci[t][v]
               : G3 ? (double)accr[t][v] + (double)accg[t][v]
                    : (double)acci[t][v];
    };

    // Shared tile: group 1 hands its partial sums to group 0 (the As buffers
    // are free once every wave is past the last chunk).
    double* xch = reinterpret_cast<double*>(As);      // [wc][v][re, im][lane]
    double sh_re[4] = {0, 0, 0, 0}, sh_im[4] = {0, 0, 0, 0};
    if (SHARED) {
        __syncthreads();
        if (GRP == 1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                xch[((wc * 4 + v) * 2 + 0) * 64 + lane] = part_re(NOWN, v);
                xch[((wc * 4 + v) * 2 + 1) * 64 + lane] = part_im(NOWN, v);
            }
        }
        __syncthreads();
        if (GRP == 0) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                sh_re[v] = part_re(NOWN, v) + xch[((wc * 4 + v) * 2 + 0) * 64 + lane];
                sh_im[v] = part_im(NOWN, v) + xch[((wc * 4 + v) * 2 + 1) * 64 + lane];
            }
        }
    }

    // Epilogue: the owned tiles, and (group 0) the shared one.
    constexpr int NOUT = NOWN + ((SHARED && GRP == 0) ? 1 : 0);
    const int col = n0 + wc * 16 + l16;
    const int s_src = col / cols_per_src;
    // Truncation: a column whose source is farther than max_radius from the
    // target stays zero (a tile can hold columns of two sources).
    bool cut = false;
    if (MODE == MODE_SOLVE && g.max_radius >= 0 && s_src < g.bs) {
        const int j = src_blk[s_src];
        int dx = i / g.Ly - j / g.Ly, dy = i % g.Ly - j % g.Ly;
        dx = dx < 0 ? -dx : dx;
        dy = dy < 0 ? -dy : dy;
        if (g.periodic) {
            dx = dx < g.Lx - dx ? dx : g.Lx - dx;
            dy = dy < g.Ly - dy ? dy : g.Ly - dy;
        }
        cut = dx + dy > g.max_radius;
    }
    const int bcol = col - s_src * cols_per_src;
    const bool own =
        (MODE != MODE_CORRECT) && !g.no_x0 && (s_src < g.bs) && (src_blk[s_src] == i);
    const dvec2* Si = S + (size_t)i * g.n_t * g.n_t;
    const cplx* Xi = X + (size_t)i * MP * ldx;
    const size_t site_off = (size_t)i * MP * ldx;
    double mdiff = 0.0, mabs = 0.0, bad = 0.0;
#pragma unroll
    for (int t = 0; t < NOUT; ++t) {
        const int tt = t < NOWN ? t0 + t : MT - 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = tt * kTile + E::row(v, lq);
            const size_t off = (size_t)row * ldx + col;
            double re = t < NOWN ? part_re(t, v) : sh_re[v];
            double im = t < NOWN ? part_im(t, v) : sh_im[v];
            // The old value is needed for the increment only (RESIDUAL always
            // needs it); sweeps that are not convergence checks skip the read.
            const bool need_old = (MODE == MODE_RESIDUAL) || g.check;
            const cplx old = need_old ? Xi[off] : cplx{0, 0};
            if (MODE == MODE_CORRECT) {
                const fvec2 r0 = R[site_off + off];
                const float yr = (float)re + r0.x, yi = (float)im + r0.y;
                reinterpret_cast<fvec2*>(out)[site_off + off] = fvec2{yr, yi};
                if (need_old)
                    mdiff = fmax(mdiff, (double)fmaxf(fabsf(yr - (float)old.x),
                                                      fabsf(yi - (float)old.y)));
                mabs = fmax(mabs, (double)fmaxf(fabsf(yr), fabsf(yi)));
                if (!(isfinite(yr) && isfinite(yi))) bad = 1.0;
            } else {
                if (cut) {
                    re = 0.0;
                    im = 0.0;
                }
                if (own && row < g.n_t) {
                    dvec2 s0;
                    if (g.x0_kind == X0_COL_T)
                        s0 = Si[(size_t)g.x0_fixed * g.n_t + row];
                    else if (g.x0_kind == X0_COL)
                        s0 = Si[(size_t)row * g.n_t + g.x0_fixed];
                    else
                        s0 = Si[(size_t)row * g.n_t + bcol];
                    re += s0.x;
                    im += s0.y;
                }
                // max-norm over real components: no overflow before a true Inf
                const double dr = re - (double)old.x, di = im - (double)old.y;
                if (MODE == MODE_SOLVE) {
                    reinterpret_cast<dvec2*>(out)[site_off + off] = dvec2{re, im};
                } else if (g.out_f64) {
                    reinterpret_cast<dvec2*>(out)[site_off + off] = dvec2{dr, di};
                } else {
                    reinterpret_cast<fvec2*>(out)[site_off + off] = fvec2{(float)dr, (float)di};
                    if (g.out2)
                        reinterpret_cast<fvec2*>(g.out2)[site_off + off] =
                            fvec2{(float)dr, (float)di};
                }
                if (need_old) mdiff = fmax(mdiff, fmax(fabs(dr), fabs(di)));
                mabs = fmax(mabs, fmax(fabs(re), fabs(im)));
                if (!(isfinite(re) && isfinite(im))) bad = 1.0;
            }
        }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        mdiff = fmax(mdiff, __shfl_xor(mdiff, m));
        mabs = fmax(mabs, __shfl_xor(mabs, m));
        bad = fmax(bad, __shfl_xor(bad, m));
    }
    if (lane == 0) {
        red[wave][0] = mdiff;
        red[wave][1] = mabs;
        red[wave][2] = bad;
    }
    __syncthreads();
    if (tid < 3) {
        double m = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) m = fmax(m, red[w][tid]);
        part[3 * blockIdx.x + tid] = m;
    }
}

template <class E, int MT, int MODE>
__global__ __launch_bounds__(kThreads, 2)
void sweep_kernel(const typename E::cplx* __restrict__ St, const dvec2* __restrict__ S,
                  const int* __restrict__ src_blk, const typename E::cplx* X, void* out,
                  const fvec2* __restrict__ R,
                  double* __restrict__ partial, SweepArgs g) {
    typedef typename E::cplx cplx;
    constexpr int MP = kTile * MT;
    constexpr int NW = kColsPerWG;
    constexpr int KC = chunk_k<E>(MT);
    constexpr int A_STRIDE = as_stride<E>(MT);
    // Two buffers each; native vector types (not HIP_vector_type) keep the
    // staging arrays in registers.
    __shared__ __attribute__((aligned(16))) cplx As[2 * A_STRIDE];   // [KC][MP] + padding
    __shared__ cplx Bs[2 * KC * NW];                                  // [KC][NW]
    __shared__ typename E::real Bd[E::gauss(MT) && E::staged_sum ? 2 * KC * NW : 2];  // br + bi
    __shared__ double red[kThreads / 64][3];

    const int tid = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int i, ct;
    tile_site_col(tile, g.ntn, g.n_sites, g.group, &i, &ct);
    if (g.sites) i = g.sites[i];
    double* part = partial + 3 * (size_t)g.part_off;
    const int n0 = ct * NW;
    const int cols_per_src = (g.x0_kind == X0_BLOCK) ? g.n_t : 1;

    int nb[4];
    site_neighbours(i, g.Lx, g.Ly, g.periodic, nb);

    // Light-cone skip (uniform per workgroup).
    if (g.lc_sweep >= 0) {
        const int s_lo = n0 / cols_per_src;
        int s_hi = (n0 + NW - 1) / cols_per_src;
        if (s_hi > g.bs - 1) s_hi = g.bs - 1;
        const int xi = i / g.Ly, yi = i - (i / g.Ly) * g.Ly;
        int dmin = 1 << 30;
        for (int s = s_lo; s <= s_hi; ++s) {
            const int j = src_blk[s];
            const int xj = j / g.Ly, yj = j - (j / g.Ly) * g.Ly;
            int dx = xi > xj ? xi - xj : xj - xi;
            int dy = yi > yj ? yi - yj : yj - yi;
            if (g.periodic) {
                dx = dx < g.Lx - dx ? dx : g.Lx - dx;
                dy = dy < g.Ly - dy ? dy : g.Ly - dy;
            }
            dmin = dmin < dx + dy ? dmin : dx + dy;
        }
        if (s_lo >= g.bs || dmin > g.lc_sweep + 1 || (g.max_radius >= 0 && dmin > g.max_radius)) {
            if (tid < 3) part[3 * blockIdx.x + tid] = 0.0;
            return;
        }
    }

    const cplx* Sti = St + (size_t)i * MP * MP;
    const cplx* Xk[4];
    for (int d = 0; d < 4; ++d) Xk[d] = nb[d] >= 0 ? X + (size_t)nb[d] * MP * g.ldx : nullptr;

    // Row group of the wave (wave-uniform; readfirstlane makes the branch a
    // scalar one).
    const int grp = __builtin_amdgcn_readfirstlane(tid >> 7);
    if (grp == 0)
        sweep_rows<E, MT, MODE, 0>(Sti, Xk, S, src_blk, X, out, R, part, g, i, n0, cols_per_src,
                                   As, Bs, Bd, red);
    else
        sweep_rows<E, MT, MODE, 1>(Sti, Xk, S, src_blk, X, out, R, part, g, i, n0, cols_per_src,
                                   As, Bs, Bd, red);
}

template <class E, int MODE>
hipError_t launch_mode(const Geom& g, const SweepArgs& a, const void* St, const double2* S,
                       const int* src_blk, const void* X, void* out, const void* R,
                       double* partial, hipStream_t st) {
    // An empty site set (the second colour of a lattice without bonds) is no
    // launch at all: it writes nothing and leaves no partials.
    if (a.n_sites * a.ntn == 0) return hipSuccess;
    dim3 grid(a.n_sites * a.ntn);
    typedef typename E::cplx cplx;
    const cplx* St_ = reinterpret_cast<const cplx*>(St);
    const cplx* X_ = reinterpret_cast<const cplx*>(X);
    const dvec2* S_ = reinterpret_cast<const dvec2*>(S);
    const fvec2* R_ = reinterpret_cast<const fvec2*>(R);
    switch (g.mt) {
#define SCD_CASE(m)                                                                         \
    case m:                                                                                 \
        hipLaunchKernelGGL((sweep_kernel<E, m, MODE>), grid, dim3(kThreads), 0, st, St_, S_, \
                           src_blk, X_, out, R_, partial, a);                              \
        return hipGetLastError();
        SCD_CASE(1) SCD_CASE(2) SCD_CASE(3) SCD_CASE(4) SCD_CASE(5) SCD_CASE(6) SCD_CASE(7)
        SCD_CASE(8) SCD_CASE(9) SCD_CASE(10) SCD_CASE(11) SCD_CASE(12) SCD_CASE(13) SCD_CASE(14)
        SCD_CASE(15) SCD_CASE(16)
#undef SCD_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_sweep_f64(const Geom& g, const SweepArgs& a, const double2* St, const double2* S,
                            const int* src_blk, const double2* X, double2* Xn, double* partial,
                            hipStream_t st) {
    return launch_mode<EngF64, MODE_SOLVE>(g, a, St, S, src_blk, X, Xn, nullptr, partial, st);
}

hipError_t launch_residual_f64(const Geom& g, const SweepArgs& a, const double2* St,
                               const double2* S, const int* src_blk, const double2* X, void* R32,
                               double* partial, hipStream_t st) {
    return launch_mode<EngF64, MODE_RESIDUAL>(g, a, St, S, src_blk, X, R32, nullptr, partial, st);
}

hipError_t launch_correct_f32(const Geom& g, const SweepArgs& a, const void* St32,
                              const int* src_blk, const void* R32, const void* D32, void* Dn32,
                              double* partial, hipStream_t st) {
    return launch_mode<EngF32, MODE_CORRECT>(g, a, St32, nullptr, src_blk, D32, Dn32, R32, partial,
                                             st);
}

}  // namespace scd

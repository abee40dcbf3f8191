// One FP64 Dyson sweep of a column block:  X'_i = X0_i + St_i^T * sum_{k in nbr(i)} X_k
// (the Dyson-series step of App. C of arXiv:1309.5994, applied to a bundle of
// unit vectors as in eq. blockedGMRESproblem), fused with the convergence
// measure of the sweep.
//
// Work decomposition (gfx950, 64-wide waves):
//  * one workgroup = one target site i and a 64-column tile of the block
//    iterate, all mp = 16*MT contour rows; 8 waves: waves 0-3 own the upper
//    row tiles and waves 4-7 the lower ones, each wave one 16-column slice, so
//    every SIMD runs all MT row tiles of one slice.
//  * K loop over contour time c in chunks of KC: the chunk of the scaled,
//    transposed site operand St_i (contiguous KC x mp complex) and the sum of
//    the (up to) four neighbour tiles X_k[c-chunk][64 cols] are staged through
//    LDS; the neighbour sum is the hopping stencil, done while staging so the
//    summed tile is never written to HBM.  Global loads of chunk k+1 are issued
//    before the MFMAs of chunk k.
//  * complex products as four real V_MFMA_F64_16X16X4_F64 per 16x16x4 block
//    (re += ar br - ai bi, im += ar bi + ai br), FP64 accumulation.
//  * epilogue adds X0 (S_j on the block's own (j, j) sub-blocks), writes X',
//    and reduces max|X' - X|, max|X'| (largest real or imaginary part) and a
//    NaN/Inf flag per workgroup.
//  * light cone: after n sweeps the iterate of source j is zero beyond
//    Manhattan distance n from j (the support argument of Sec. IV.D); a tile
//    whose sources are all farther than n+1 from site i is skipped (its output
//    stays zero).
#include "internal.h"

namespace scd {
namespace {

constexpr int kThreads = 512;

template <int MT, int KC>
__global__ __launch_bounds__(kThreads)
void sweep_f64_kernel(const double2* __restrict__ St, const double2* __restrict__ S,
                      const int* __restrict__ src_blk, const double2* __restrict__ X,
                      double2* __restrict__ Xn, double* __restrict__ partial, SweepArgs g) {
    constexpr int MP = kTile * MT;
    constexpr int NW = kColsPerWG;
    constexpr int MH = (MT + 1) / 2;                 // row tiles of the upper wave group
    constexpr int A_ELEMS = KC * MP;
    constexpr int A_PER = (A_ELEMS + kThreads - 1) / kThreads;
    constexpr int B_ELEMS = KC * NW;
    constexpr int B_PER = (B_ELEMS + kThreads - 1) / kThreads;
    static_assert(MP % KC == 0, "k chunk must divide the padded contour length");

    static_assert(B_ELEMS % kThreads == 0, "B chunk must be a whole number of passes");
    // Native vector types (not HIP_vector_type) keep the staging arrays in registers.
    __shared__ dvec2 As[A_PER * kThreads];   // [KC][MP] + padding of the last pass
    __shared__ dvec2 Bs[B_ELEMS];            // [KC][NW]
    __shared__ double red[kThreads / 64][3];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int grp = wave >> 2;
    const int wc = wave & 3;
    const int l16 = lane & 15;
    const int lq = lane >> 4;

    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int i, ct;
    tile_site_col(tile, g.ntn, g.n_r, g.group, &i, &ct);
    const int n0 = ct * NW;
    const int ldx = g.ldx;

    int nb[4];
    site_neighbours(i, g.Lx, g.Ly, g.periodic, nb);

    // Light-cone skip (uniform per workgroup).
    if (g.lc_sweep >= 0) {
        const int s_lo = n0 / g.n_t;
        int s_hi = (n0 + NW - 1) / g.n_t;
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
        if (s_lo >= g.bs || dmin > g.lc_sweep + 1) {
            if (tid == 0) {
                partial[3 * blockIdx.x + 0] = 0.0;
                partial[3 * blockIdx.x + 1] = 0.0;
                partial[3 * blockIdx.x + 2] = 0.0;
            }
            return;
        }
    }

    const dvec2* Sti = reinterpret_cast<const dvec2*>(St) + (size_t)i * MP * MP;
    const dvec2* Xk[4];
    for (int d = 0; d < 4; ++d)
        Xk[d] = nb[d] >= 0 ? reinterpret_cast<const dvec2*>(X) + (size_t)nb[d] * MP * ldx : nullptr;

    dvec4 accr[MH], acci[MH];
#pragma unroll
    for (int t = 0; t < MH; ++t) {
        accr[t] = dvec4{0.0, 0.0, 0.0, 0.0};
        acci[t] = dvec4{0.0, 0.0, 0.0, 0.0};
    }
    const int t0 = grp ? MH : 0;
    const int ntile = grp ? MT - MH : MH;

    dvec2 ra[A_PER];
    dvec2 rb[B_PER][4];

    // Staging of one K chunk: global -> registers (issued a chunk ahead) and
    // registers -> LDS.  Threads past the end of the A chunk re-load its last
    // element into LDS padding, so no lane is predicated off.
#define SCD_GLOAD(k0)                                                                  \
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
                rb[r][d] = Xk[d] ? Xk[d][off] : dvec2{0.0, 0.0};                       \
        }                                                                              \
    } while (0)
#define SCD_LSTORE()                                                                   \
    do {                                                                               \
        _Pragma("unroll") for (int r = 0; r < A_PER; ++r) As[tid + r * kThreads] = ra[r]; \
        _Pragma("unroll") for (int r = 0; r < B_PER; ++r) {                            \
            Bs[tid + r * kThreads] = (rb[r][0] + rb[r][1]) + (rb[r][2] + rb[r][3]);    \
        }                                                                              \
    } while (0)

    SCD_GLOAD(0);
    for (int k0 = 0; k0 < MP; k0 += KC) {
        __syncthreads();
        SCD_LSTORE();
        __syncthreads();
        if (k0 + KC < MP) SCD_GLOAD(k0 + KC);
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int kr = 4 * s + lq;
            const dvec2 b = Bs[kr * NW + wc * 16 + l16];
            dvec2 a[MH];
#pragma unroll
            for (int t = 0; t < MH; ++t)
                if (t < ntile) a[t] = As[kr * MP + (t0 + t) * kTile + l16];
#pragma unroll
            for (int t = 0; t < MH; ++t) {
                if (t < ntile) {
                    accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b.x, accr[t], 0, 0, 0);
                    acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].x, b.y, acci[t], 0, 0, 0);
                }
            }
#pragma unroll
            for (int t = 0; t < MH; ++t) {
                if (t < ntile) {
                    accr[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[t].y, b.y, accr[t], 0, 0, 0);
                    acci[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t].y, b.x, acci[t], 0, 0, 0);
                }
            }
        }
    }

    // Epilogue: X' = acc + X0, convergence partials.
    const int col = n0 + wc * 16 + l16;
    const int s_src = col / g.n_t;
    const int bcol = col - s_src * g.n_t;
    const bool own = (s_src < g.bs) && (src_blk[s_src] == i);
    const double2* Si = S + (size_t)i * g.n_t * g.n_t;
    const double2* Xi = X + (size_t)i * MP * ldx;
    double2* Xni = Xn + (size_t)i * MP * ldx;
    double mdiff = 0.0, mabs = 0.0, bad = 0.0;
#pragma unroll
    for (int t = 0; t < MH; ++t) {
        if (t < ntile) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                // V_MFMA_F64_16X16X4_F64 result: element v of lane l is row 4 v + l / 16, column l % 16.
                const int row = (t0 + t) * kTile + 4 * v + lq;
                double re = accr[t][v], im = acci[t][v];
                if (own && row < g.n_t) {
                    const double2 s0 = Si[(size_t)row * g.n_t + bcol];
                    re += s0.x;
                    im += s0.y;
                }
                const size_t off = (size_t)row * ldx + col;
                const double2 old = Xi[off];
                Xni[off] = make_double2(re, im);
                // max-norm over real components: no overflow before a true Inf
                mdiff = fmax(mdiff, fmax(fabs(re - old.x), fabs(im - old.y)));
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
        partial[3 * blockIdx.x + tid] = m;
    }
#undef SCD_GLOAD
#undef SCD_LSTORE
}

template <int MT>
hipError_t launch_mt(const SweepArgs& a, dim3 grid, const double2* St, const double2* S,
                     const int* src_blk, const double2* X, double2* Xn, double* partial,
                     hipStream_t st) {
    constexpr int KC = (MT % 2 == 0) ? 8 : 16;   // keep MP % KC == 0 and LDS modest
    hipLaunchKernelGGL((sweep_f64_kernel<MT, KC>), grid, dim3(kThreads), 0, st, St, S, src_blk, X,
                       Xn, partial, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sweep_f64(const Geom& g, const SweepArgs& a, const double2* St, const double2* S,
                            const int* src_blk, const double2* X, double2* Xn, double* partial,
                            hipStream_t st) {
    dim3 grid(g.n_r * a.ntn);
    switch (g.mt) {
#define SCD_CASE(m) \
    case m: return launch_mt<m>(a, grid, St, S, src_blk, X, Xn, partial, st);
        SCD_CASE(1) SCD_CASE(2) SCD_CASE(3) SCD_CASE(4) SCD_CASE(5) SCD_CASE(6) SCD_CASE(7)
        SCD_CASE(8) SCD_CASE(9) SCD_CASE(10) SCD_CASE(11) SCD_CASE(12) SCD_CASE(13) SCD_CASE(14)
        SCD_CASE(15) SCD_CASE(16)
#undef SCD_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace scd

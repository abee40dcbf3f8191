// FP32-accuracy correction sweep of the mixed-precision refinement on the
// BF16 matrix cores (BF16x3 split products):
//
//     D'_i = R_i + St_i^T * sum_{k in nbr(i)} D_k        (complex64 in HBM)
//
// the CORRECT-mode sweep of sweep.hip with its products split in the manner
// of Henry, Tang and Heinecke (ARITH 2019): every FP32 value x is carried as
// x_hi = bf16(x), x_lo = bf16(x - x_hi), and a real product as
// a_hi b_hi + a_hi b_lo + a_lo b_hi with FP32 accumulation (relative error
// near 2^-16 per product).  Complex products use the four-product form
// re += ar br + ai (-bi), im += ar bi + ai br, so one complex block product
// is 12 MFMAs V_MFMA_F32_16X16X32_BF16.  (The three-product form saves MFMAs
// but needs six operand planes per row tile instead of four; the kernel is
// bound by those LDS fragment reads, not by the matrix cores.)
//
// Operands:
//  * the site operand is precomputed once per solve (launch_bf3_operand):
//    per site four bf16 planes (hi/lo of ar, ai) of St_i^T, i.e.
//    [plane][row a][k], k contiguous and padded with zeros to a multiple of
//    32, so that a lane's eight consecutive k of one row are 16 bytes;
//  * the neighbour sum is split into six planes (hi/lo of br, bi, -bi),
//    [plane][column][k], while it is staged.
//
// Work decomposition: as the FP32/FP64 sweeps (one workgroup = one target
// site and a 32-column tile, 4 waves: two row groups x two 16-column slices,
// the last row tile of an odd MT shared by the two groups over alternate
// chunks).  One chunk = one MFMA k-step of 32 contour points.  The St chunk
// reaches LDS by DMA (global_load_lds_dwordx4; no staging registers).  An LDS
// row of a plane holds the chunk's 32 bf16 of one row as four 16-byte units,
// unit j of row r stored in slot j ^ ((r >> 2) & 3), so that the 16 rows one
// fragment read touches fall on distinct banks; the neighbour tiles of the
// next chunk are loaded into registers while the current chunk is multiplied.
#include "internal.h"

namespace scd {
namespace {

constexpr int kThreadsB = 256;
constexpr int kKB = 32;                  // contour points per chunk (one MFMA k-step)
constexpr int kRowB = kKB;               // LDS row of one plane, in bf16 (64 bytes)
constexpr int kPlanesA = 4;              // ar hi, ar lo, ai hi, ai lo
constexpr int kPlanesB = 6;              // br hi/lo, bi hi/lo, -bi hi/lo

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) const void* glob_ptr;
typedef __attribute__((address_space(3))) void* lds_ptr;

__device__ __forceinline__ fvec4 mma_bf16(bf16x8 a, bf16x8 b, fvec4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// x = hi + lo in bf16 (round to nearest even both times).
__device__ __forceinline__ void split_bf16(float x, __bf16* hi, __bf16* lo) {
    *hi = (__bf16)x;
    *lo = (__bf16)(x - (float)*hi);
}

// Padded K of an MT-tile operand.
__host__ __device__ constexpr int bf3_kpad(int mt) { return (kTile * mt + kKB - 1) / kKB * kKB; }

template <int MT, int GRP>
__device__ __forceinline__ void bf3_rows(const __bf16* __restrict__ Ai,
                                         const fvec2* const (&Xk)[4],
                                         const int* __restrict__ src_blk, const fvec2* X,
                                         fvec2* out, const fvec2* __restrict__ R, double* part,
                                         const SweepArgs& g, int i, int n0,
                                         __bf16* As, __bf16* Bsp, double (*red)[3]) {
    constexpr int MP = kTile * MT;
    constexpr int KP = bf3_kpad(MT);
    constexpr int NW = kColsPerWG;
    constexpr int NOWN = MT / 2;
    constexpr bool SHARED = (MT % 2) != 0;
    constexpr int NA = NOWN + (SHARED ? 1 : 0);
    // St chunk: kPlanesA x MP rows x 4 units of 16 bytes.
    constexpr int A_UNITS = kPlanesA * MP * 4;
    constexpr int A_PER = (A_UNITS + kThreadsB - 1) / kThreadsB;
    constexpr int B_ELEMS = kKB * NW;                   // 1024 per chunk
    constexpr int B_PER = B_ELEMS / kThreadsB;          // 4: one column, 4 consecutive k
    static_assert(B_PER == 4, "each thread stages four consecutive contour points");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wc = wave & 1;
    const int l16 = lane & 15;
    const int lq = lane >> 4;
    const int ldx = g.ldx;
    const int t0 = GRP * NOWN;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);

    fvec4 acc[NA][2];   // re, im
#pragma unroll
    for (int t = 0; t < NA; ++t)
#pragma unroll
        for (int q = 0; q < 2; ++q) acc[t][q] = fvec4{0, 0, 0, 0};

    // Neighbour staging: thread -> column bc, contour points 4 bq .. 4 bq + 3.
    const int bc = tid % NW, bq = tid / NW;
    fvec2 rb[B_PER][4];

    auto load_b = [&](int k0) __attribute__((always_inline)) {
#pragma unroll
        for (int j = 0; j < B_PER; ++j) {
            const int k = k0 + 4 * bq + j;
            const size_t off = (size_t)k * ldx + n0 + bc;
#pragma unroll
            for (int d = 0; d < 4; ++d)
                rb[j][d] = (Xk[d] && k < MP) ? Xk[d][off] : fvec2{0, 0};
        }
    };
    auto dma_a = [&](int k0) __attribute__((always_inline)) {
        const char* base = reinterpret_cast<const char*>(Ai);
#pragma unroll
        for (int r = 0; r < A_PER; ++r) {
            const int blk = r * (kThreadsB / 64) + wave_u;
            int u = blk * 64 + lane;
            u = u < A_UNITS ? u : A_UNITS - 1;
            const int pr = u >> 2, j = u & 3;                // (plane, row), slot in row
            const int jd = j ^ ((pr >> 2) & 3);              // data unit held by the slot
            const size_t src = ((size_t)pr * KP + k0 + 8 * jd) * sizeof(__bf16);
            __builtin_amdgcn_global_load_lds((glob_ptr)(base + src),
                                             (lds_ptr)(reinterpret_cast<char*>(As) + blk * 1024),
                                             16, 0, 0);
        }
    };
    auto store_b = [&]() __attribute__((always_inline)) {
        bf16x4 pl[kPlanesB];
#pragma unroll
        for (int j = 0; j < B_PER; ++j) {
            const fvec2 v = (rb[j][0] + rb[j][1]) + (rb[j][2] + rb[j][3]);
            __bf16 h, l;
            split_bf16(v.x, &h, &l);
            pl[0][j] = h;
            pl[1][j] = l;
            split_bf16(v.y, &h, &l);
            pl[2][j] = h;
            pl[3][j] = l;
            pl[4][j] = -h;     // rounding is symmetric: split(-x) = -split(x)
            pl[5][j] = -l;
        }
        // contour points 4 bq .. 4 bq + 3 = half (bq & 1) of unit bq >> 1
        const int slot = ((bq >> 1) ^ ((bc >> 2) & 3)) * 8 + (bq & 1) * 4;
#pragma unroll
        for (int p = 0; p < kPlanesB; ++p)
            *reinterpret_cast<bf16x4*>(Bsp + ((size_t)p * NW + bc) * kRowB + slot) = pl[p];
    };

    // Single-buffered LDS, two barriers per chunk (two workgroups share a CU
    // and cover each other's barriers).
    load_b(0);
    for (int k0 = 0, c = 0; k0 < KP; k0 += kKB, ++c) {
        __syncthreads();                 // every wave done with the previous chunk
        dma_a(k0);
        store_b();
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        __syncthreads();                 // chunk c in LDS
        if (k0 + kKB < KP) load_b(k0 + kKB);
        // Fragments: lane (l16, lq) holds row / column l16 and contour points
        // 8 lq .. 8 lq + 7 of the chunk.
        const bool sh = SHARED && ((c & 1) == GRP);
        const int nt = NOWN + (sh ? 1 : 0);
        // rows / columns of a fragment are 16-aligned, so their swizzle is
        // that of l16
        const int fslot = 8 * (lq ^ ((l16 >> 2) & 3));
        bf16x8 b[kPlanesB];
#pragma unroll
        for (int p = 0; p < kPlanesB; ++p)
            b[p] = *reinterpret_cast<const bf16x8*>(
                Bsp + ((size_t)p * NW + wc * 16 + l16) * kRowB + fslot);
#pragma unroll
        for (int t = 0; t < NA; ++t) {
            if (t < nt) {
                const int tt = t < NOWN ? t0 + t : MT - 1;
                bf16x8 a[kPlanesA];
#pragma unroll
                for (int p = 0; p < kPlanesA; ++p)
                    a[p] = *reinterpret_cast<const bf16x8*>(
                        As + ((size_t)p * MP + tt * kTile + l16) * kRowB + fslot);
                // x y ~ x_lo y_hi + x_hi y_lo + x_hi y_hi, small terms first;
                // plane 2q is hi, 2q + 1 lo.
#define SCD_X3(acc_, ia, ib)                                                       \
    acc_ = mma_bf16(a[(ia) + 1], b[(ib)], acc_);                                   \
    acc_ = mma_bf16(a[(ia)], b[(ib) + 1], acc_);                                   \
    acc_ = mma_bf16(a[(ia)], b[(ib)], acc_)
                SCD_X3(acc[t][0], 0, 0);   // re += ar br
                SCD_X3(acc[t][0], 2, 4);   // re += ai (-bi)
                SCD_X3(acc[t][1], 0, 2);   // im += ar bi
                SCD_X3(acc[t][1], 2, 0);   // im += ai br
#undef SCD_X3
            }
        }
    }

    // Complex partial sums of tile t, element v.
    auto part_re = [&](int t, int v) -> float { return acc[t][0][v]; };
    auto part_im = [&](int t, int v) -> float { return acc[t][1][v]; };

    // Shared tile: group 1 hands its partial sums to group 0 through LDS.
    float sh_re[4] = {0, 0, 0, 0}, sh_im[4] = {0, 0, 0, 0};
    if (SHARED) {
        float* xch = reinterpret_cast<float*>(As);    // [wc][v][re, im][lane]
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

    // Epilogue: D' = R + y; partials max|D' - D| (checked sweeps), max|D'|,
    // NaN/Inf flag.  V_MFMA_F32_16X16X32_BF16 result: element v of lane l is
    // row 4 (l/16) + v, column l%16.
    constexpr int NOUT = NOWN + ((SHARED && GRP == 0) ? 1 : 0);
    const int col = n0 + wc * 16 + l16;
    const fvec2* Xi = X + (size_t)i * MP * ldx;
    const size_t site_off = (size_t)i * MP * ldx;
    double mdiff = 0.0, mabs = 0.0, bad = 0.0;
#pragma unroll
    for (int t = 0; t < NOUT; ++t) {
        const int tt = t < NOWN ? t0 + t : MT - 1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int row = tt * kTile + 4 * lq + v;
            const size_t off = (size_t)row * ldx + col;
            const float re = t < NOWN ? part_re(t, v) : sh_re[v];
            const float im = t < NOWN ? part_im(t, v) : sh_im[v];
            const fvec2 r0 = R[site_off + off];
            const float yr = re + r0.x, yi = im + r0.y;
            // Red-black sweeps update D in place: read the old value first.
            if (g.check) {
                const fvec2 old = Xi[off];
                mdiff = fmax(mdiff, (double)fmaxf(fabsf(yr - old.x), fabsf(yi - old.y)));
            }
            out[site_off + off] = fvec2{yr, yi};
            mabs = fmax(mabs, (double)fmaxf(fabsf(yr), fabsf(yi)));
            if (!(isfinite(yr) && isfinite(yi))) bad = 1.0;
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
        for (int w = 0; w < kThreadsB / 64; ++w) m = fmax(m, red[w][tid]);
        part[3 * blockIdx.x + tid] = m;
    }
}

template <int MT>
__global__ __launch_bounds__(kThreadsB, 2)
void bf3_kernel(const __bf16* __restrict__ Abf, const int* __restrict__ src_blk,
                const fvec2* X, fvec2* out, const fvec2* __restrict__ R,
                double* __restrict__ partial, SweepArgs g) {
    constexpr int MP = kTile * MT;
    constexpr int KP = bf3_kpad(MT);
    constexpr int NW = kColsPerWG;
    constexpr int A_UNITS = kPlanesA * MP * 4;
    constexpr int A_BYTES = (A_UNITS + kThreadsB - 1) / kThreadsB * kThreadsB * 16;
    static_assert(A_BYTES >= 2 * 4 * 2 * 64 * 4, "As also carries the shared tile's sums");
    __shared__ __attribute__((aligned(16))) __bf16 As[A_BYTES / 2];
    __shared__ __attribute__((aligned(16))) __bf16 Bsp[kPlanesB * NW * kRowB];
    __shared__ double red[kThreadsB / 64][3];

    const int tid = threadIdx.x;
    const int tile = xcd_remap(blockIdx.x, gridDim.x);
    int i, ct;
    tile_site_col(tile, g.ntn, g.n_sites, g.group, &i, &ct);
    if (g.sites) i = g.sites[i];
    double* part = partial + 3 * (size_t)g.part_off;
    const int n0 = ct * NW;
    const int cols_per_src = (g.x0_kind == X0_BLOCK) ? g.n_t : 1;

    // Light-cone skip (uniform per workgroup), as in the FP64/FP32 sweeps.
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
        if (s_lo >= g.bs || dmin > g.lc_sweep + 1) {
            if (tid < 3) part[3 * blockIdx.x + tid] = 0.0;
            return;
        }
    }

    int nb[4];
    site_neighbours(i, g.Lx, g.Ly, g.periodic, nb);
    const __bf16* Ai = Abf + (size_t)i * kPlanesA * MP * KP;
    const fvec2* Xk[4];
    for (int d = 0; d < 4; ++d) Xk[d] = nb[d] >= 0 ? X + (size_t)nb[d] * MP * g.ldx : nullptr;

    const int grp = __builtin_amdgcn_readfirstlane(tid >> 7);
    if (grp == 0)
        bf3_rows<MT, 0>(Ai, Xk, src_blk, X, out, R, part, g, i, n0, As, Bsp, red);
    else
        bf3_rows<MT, 1>(Ai, Xk, src_blk, X, out, R, part, g, i, n0, As, Bsp, red);
}

// Four bf16 planes per site from St (complex128 [site][c][a], mp x mp):
// plane[p][a][k] for k < mp (hi/lo of Re and Im of St_i[k][a]), zero for
// mp <= k < kp.
__global__ __launch_bounds__(256)
void bf3_operand_kernel(const dvec2* __restrict__ St, int n_sites, int mp, int kp,
                        __bf16* __restrict__ out) {
    const size_t per = (size_t)mp * kp;
    const size_t n = (size_t)n_sites * per;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t site = e / per, rem = e - site * per;
        const int a = (int)(rem / kp), k = (int)(rem - (size_t)a * kp);
        float xr = 0.0f, xi = 0.0f;
        if (k < mp) {
            const dvec2 v = St[(site * mp + k) * mp + a];
            xr = (float)v.x;
            xi = (float)v.y;
        }
        __bf16* o = out + site * kPlanesA * per + rem;
        __bf16 h, l;
        split_bf16(xr, &h, &l);
        o[0 * per] = h;
        o[1 * per] = l;
        split_bf16(xi, &h, &l);
        o[2 * per] = h;
        o[3 * per] = l;
    }
}

}  // namespace

size_t bf3_operand_bytes(const Geom& g) {
    return (size_t)g.n_r * kPlanesA * g.mp * bf3_kpad(g.mt) * sizeof(__bf16);
}

hipError_t launch_bf3_operand(const Geom& g, const double2* St, void* out, hipStream_t st) {
    hipLaunchKernelGGL(bf3_operand_kernel, dim3(4096), dim3(256), 0, st,
                       reinterpret_cast<const dvec2*>(St), g.n_r, g.mp, bf3_kpad(g.mt),
                       reinterpret_cast<__bf16*>(out));
    return hipGetLastError();
}

hipError_t launch_correct_bf3(const Geom& g, const SweepArgs& a, const void* Abf,
                              const int* src_blk, const void* R32, const void* D32, void* Dn32,
                              double* partial, hipStream_t st) {
    if (a.n_sites * a.ntn == 0) return hipSuccess;     // empty colour: nothing to update
    const dim3 grid(a.n_sites * a.ntn);
    const __bf16* A_ = reinterpret_cast<const __bf16*>(Abf);
    const fvec2* X_ = reinterpret_cast<const fvec2*>(D32);
    fvec2* O_ = reinterpret_cast<fvec2*>(Dn32);
    const fvec2* R_ = reinterpret_cast<const fvec2*>(R32);
    switch (g.mt) {
#define SCD_CASE(m)                                                                          \
    case m:                                                                                  \
        hipLaunchKernelGGL((bf3_kernel<m>), grid, dim3(kThreadsB), 0, st, A_, src_blk, X_,   \
                           O_, R_, partial, a);                                              \
        return hipGetLastError();
        SCD_CASE(1) SCD_CASE(2) SCD_CASE(3) SCD_CASE(4) SCD_CASE(5) SCD_CASE(6) SCD_CASE(7)
        SCD_CASE(8) SCD_CASE(9) SCD_CASE(10) SCD_CASE(11) SCD_CASE(12) SCD_CASE(13) SCD_CASE(14)
        SCD_CASE(15) SCD_CASE(16)
#undef SCD_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace scd

// Device side of the batched preconditioned GMRES (App. C of arXiv:1309.5994):
// the per-column Gram-Schmidt passes over the Krylov basis, the Givens-rotated
// Hessenberg least-squares problem of every column, and the solution update.
//
// Vectors are block iterates [N_r][mp][ldx] complex128: rows are (site,
// contour row), columns (source, contour column).  Every column is its own
// GMRES problem (one unit vector of eq. blockedGMRESproblem), so every
// reduction runs down the rows of one column.  The batched matvec is the sweep
// kernel (sweep.hip) with X0 left out.
//
// Basis vectors are stored unnormalised, q_i = sig_i v_i with one scale per
// column: the operator acts on rows only, so it commutes with a per-column
// scale and no pass over HBM is spent on normalising.
//
// Streaming passes (HBM-bound): one 16-byte complex per thread and row, each
// wave 64 consecutive columns (1 KB per row), four waves on interleaved rows:
//   DOTS          p_i = sum_rows conj(q_i) x,            x = ws w
//   PROJ_DOTS     x = ws w - sum_i c_i q_i (registers);  p_i = sum_rows conj(q_i) x
//   UPDATE_NORM   x = ws w - sum_i c_i q_i; write x;     |x|^2
//   NORM          |w|^2
//   UPDATE        w = w - sum_i c_i q_i (the solution update, c = -y)
// with i < k.  Classical Gram-Schmidt applied twice is DOTS (h1), PROJ_DOTS
// with c = h1 (h2, the dots of the once-projected vector, which is not
// stored) and UPDATE_NORM with c = h1 + h2 from the matvec output again: the
// same projections as two stored passes, with one vector less moved per step
// and a read-only middle pass.  Krylov vectors are read with non-temporal
// loads (streamed once per pass, no reuse in the caches).  A workgroup covers 64 columns and one chunk of rows; partial
// sums go to [chunk][i][column] and their consumer adds the chunks in order,
// so results do not depend on scheduling (no atomics).
#include "internal.h"

namespace scd {
namespace {

constexpr int kGsThreads = 256;
constexpr int kGsCols = 64;

__device__ inline dvec2 cmul(dvec2 a, dvec2 b) {
    return dvec2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// conj(a) * b
__device__ inline dvec2 cmulc(dvec2 a, dvec2 b) {
    return dvec2{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

template <int KB, bool UPDATE, bool DOTS, bool NORM, bool WRITE>
__global__ __launch_bounds__(kGsThreads)
void gs_kernel(GsPass p) {
    __shared__ dvec2 red[kGsThreads];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int c = blockIdx.x * kGsCols + lane;
    const bool live = c < p.ldx;
    const int cc = live ? c : p.ldx - 1;
    const dvec2* Q = reinterpret_cast<const dvec2*>(p.Q);
    dvec2* w = reinterpret_cast<dvec2*>(p.w);
    const dvec2* coef = reinterpret_cast<const dvec2*>(p.coef);
    const dvec2* coef2 = reinterpret_cast<const dvec2*>(p.coef2);

    // The column scales enter outside the row loop: the update uses
    // c_i sig_i, the dots are sig_i sum conj(v_i) x.
    dvec2 cf[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) {
        cf[i] = dvec2{0.0, 0.0};
        if (UPDATE && i < p.k) {
            for (int q = 0; q < p.coef_parts; ++q)
                cf[i] += coef[(size_t)q * p.coef_pstride + (size_t)i * p.ldx + cc];
            if (coef2)
                for (int q = 0; q < p.coef_parts; ++q)
                    cf[i] += coef2[(size_t)q * p.coef_pstride + (size_t)i * p.ldx + cc];
            cf[i] *= p.sig[(size_t)i * p.ldx + cc];
        }
    }
    const double ws = p.wsig ? p.wsig[cc] : 1.0;
    dvec2 acc[KB];
#pragma unroll
    for (int i = 0; i < KB; ++i) acc[i] = dvec2{0.0, 0.0};
    double nrm = 0.0;

    int r0 = blockIdx.y * p.chunk_rows;
    int r1 = min(p.rows, r0 + p.chunk_rows);
    if (p.radius >= 0) {
        // Workgroup-uniform: nearest (site of the chunk, source of the strip) pair.
        const int c_lo = blockIdx.x * kGsCols;
        const int s_lo = c_lo / p.n_t;
        const int s_hi = min((c_lo + kGsCols - 1) / p.n_t, p.bs - 1);
        const int i_lo = r0 / p.mp, i_hi = (r1 - 1) / p.mp;
        int dmin = 1 << 30;
        for (int s = s_lo; s <= s_hi; ++s) {
            const int j = p.src_blk[s];
            const int xj = j / p.Ly, yj = j - (j / p.Ly) * p.Ly;
            for (int i = i_lo; i <= i_hi; ++i) {
                const int xi = i / p.Ly, yi = i - (i / p.Ly) * p.Ly;
                int dx = xi > xj ? xi - xj : xj - xi;
                int dy = yi > yj ? yi - yj : yj - yi;
                if (p.periodic) {
                    dx = min(dx, p.Lx - dx);
                    dy = min(dy, p.Ly - dy);
                }
                dmin = min(dmin, dx + dy);
            }
        }
        if (s_lo >= p.bs || dmin > p.radius) r1 = r0;    // all rows zero: partials only
    }
    for (int r = r0 + wv; r < r1; r += 4) {
        const size_t off = (size_t)r * p.ldx + cc;
        dvec2 x = __builtin_nontemporal_load(&w[off]) * ws;
        dvec2 v[KB];
#pragma unroll
        for (int i = 0; i < KB; ++i)
            v[i] = i < p.k ? __builtin_nontemporal_load(&Q[(size_t)i * p.qstride + off])
                           : dvec2{0.0, 0.0};
        if (UPDATE) {
#pragma unroll
            for (int i = 0; i < KB; ++i) x -= cmul(cf[i], v[i]);
        }
        if (DOTS) {
#pragma unroll
            for (int i = 0; i < KB; ++i) acc[i] += cmulc(v[i], x);
        }
        if (NORM) nrm += x.x * x.x + x.y * x.y;
        if (WRITE && live) __builtin_nontemporal_store(x, &w[off]);   // read back from HBM next pass
    }
    if (DOTS) {
#pragma unroll
        for (int i = 0; i < KB; ++i)
            if (i < p.k) acc[i] *= p.sig[(size_t)i * p.ldx + cc];
    }

    // Add the four waves' partials, one basis index at a time through LDS.
    if (DOTS) {
        dvec2* pd = reinterpret_cast<dvec2*>(p.pdot) + (size_t)blockIdx.y * kMaxBasis * p.ldx;
#pragma unroll
        for (int i = 0; i < KB; ++i) {
            if (i < p.k) {       // uniform over the workgroup
                red[threadIdx.x] = acc[i];
                __syncthreads();
                if (wv == 0 && live)
                    pd[(size_t)i * p.ldx + c] =
                        red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
                __syncthreads();
            }
        }
    }
    if (NORM) {
        red[threadIdx.x] = dvec2{nrm, 0.0};
        __syncthreads();
        if (wv == 0 && live)
            p.pnorm[(size_t)blockIdx.y * p.ldx + c] =
                red[lane].x + red[64 + lane].x + red[128 + lane].x + red[192 + lane].x;
    }
}

// Per-workgroup (max, 1, bad) triple of a per-column quantity, for the
// convergence reduction the sweeps use as well.
__device__ inline void block_max_triple(double v, double bad, double* part) {
    __shared__ double rv[256], rb[256];
    rv[threadIdx.x] = v;
    rb[threadIdx.x] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            rv[threadIdx.x] = fmax(rv[threadIdx.x], rv[threadIdx.x + s]);
            rb[threadIdx.x] = fmax(rb[threadIdx.x], rb[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = rv[0];
        part[3 * blockIdx.x + 1] = 1.0;
        part[3 * blockIdx.x + 2] = rb[0];
    }
}

// One Arnoldi step's Hessenberg column for every column c of the block, or
// (d < 0) the start of a cycle.
//
// The basis is built with T = St^T N (the Dyson-series operator S D), whose
// Arnoldi relation T Q_k = Q_{k+1} H_T gives for the preconditioned system
// matrix M = I - S D:  M Q_k = Q_{k+1} (I_{k+1,k} - H_T).  Column d of that
// Hessenberg matrix is delta_{jd} - h_j (j <= d) and -h_{d+1,d}; the earlier
// rotations are applied to it, a new one annihilates its subdiagonal, and the
// rotated right-hand side g gives the residual 2-norm |g_{d+1}| (App. C, step
// 3, by Givens rotations instead of a fresh least-squares solve).
__global__ __launch_bounds__(256)
void givens_kernel(GivensArgs a) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    double ratio = 0.0, bad = 0.0;
    if (c < a.ldx) {
        const size_t L = a.ldx;
        double nn = 0.0;
        for (int ch = 0; ch < a.nch; ++ch) nn += a.pn[(size_t)ch * L + c];
        const double hn = sqrt(nn);
        dvec2* R = reinterpret_cast<dvec2*>(a.R);
        dvec2* sn = reinterpret_cast<dvec2*>(a.sn);
        dvec2* gv = reinterpret_cast<dvec2*>(a.gv);
        double res;
        if (a.d < 0) {
            a.sig[c] = hn > 0.0 ? 1.0 / hn : 0.0;
            gv[c] = dvec2{hn, 0.0};
            res = hn;
        } else {
            const int d = a.d;
            const dvec2* pa = reinterpret_cast<const dvec2*>(a.pa);
            const dvec2* pb = reinterpret_cast<const dvec2*>(a.pb);
            // Column d of I - H_T into R[:, d] (row j at R[(j * kMaxBasis + d) L + c]).
            for (int j = 0; j <= d; ++j) {
                dvec2 h = dvec2{0.0, 0.0};
                for (int ch = 0; ch < a.nch; ++ch) {
                    const size_t o = ((size_t)ch * kMaxBasis + j) * L + c;
                    h += pa[o] + pb[o];
                }
                R[((size_t)j * kMaxBasis + d) * L + c] = dvec2{(j == d ? 1.0 : 0.0) - h.x, -h.y};
            }
            // Earlier rotations.
            for (int j = 0; j < d; ++j) {
                const double cj = a.cs[(size_t)j * L + c];
                const dvec2 sj = sn[(size_t)j * L + c];
                const dvec2 x = R[((size_t)j * kMaxBasis + d) * L + c];
                const dvec2 y = R[((size_t)(j + 1) * kMaxBasis + d) * L + c];
                R[((size_t)j * kMaxBasis + d) * L + c] = x * cj + cmul(sj, y);
                R[((size_t)(j + 1) * kMaxBasis + d) * L + c] =
                    y * cj - cmul(dvec2{sj.x, -sj.y}, x);
            }
            // New rotation [c s; -conj(s) c] taking (x, b) to (r, 0), b = -hn real.
            const dvec2 x = R[((size_t)d * kMaxBasis + d) * L + c];
            const double b = -hn;
            const double ax = sqrt(x.x * x.x + x.y * x.y);
            double cr;
            dvec2 sr, r;
            if (ax == 0.0) {
                cr = 0.0;
                sr = dvec2{1.0, 0.0};
                r = dvec2{b, 0.0};
                if (b == 0.0) {
                    cr = 1.0;
                    sr = dvec2{0.0, 0.0};
                }
            } else {
                const double nu = sqrt(ax * ax + b * b);
                const dvec2 ph = x * (1.0 / ax);
                cr = ax / nu;
                sr = ph * (b / nu);
                r = ph * nu;
            }
            a.cs[(size_t)d * L + c] = cr;
            sn[(size_t)d * L + c] = sr;
            R[((size_t)d * kMaxBasis + d) * L + c] = r;
            const dvec2 gd = gv[(size_t)d * L + c];
            gv[(size_t)d * L + c] = gd * cr;
            const dvec2 g1 = cmul(dvec2{-sr.x, sr.y}, gd);
            gv[(size_t)(d + 1) * L + c] = g1;
            a.sig[(size_t)(d + 1) * L + c] = hn > 0.0 ? 1.0 / hn : 0.0;
            res = sqrt(g1.x * g1.x + g1.y * g1.y);
        }
        const double ref = a.x0n[c];
        ratio = ref > 0.0 ? res / ref : 0.0;
        if (!isfinite(res)) bad = 1.0;
    }
    block_max_triple(ratio, bad, a.part);
}

// y = R^-1 g over the first k rotated rows; stores c = -y for the UPDATE pass.
__global__ __launch_bounds__(256)
void gmres_solve_kernel(const double2* __restrict__ R_, const double2* __restrict__ gv_,
                        double2* __restrict__ y_, int k, int ldx) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ldx) return;
    const size_t L = ldx;
    const dvec2* R = reinterpret_cast<const dvec2*>(R_);
    const dvec2* gv = reinterpret_cast<const dvec2*>(gv_);
    dvec2* y = reinterpret_cast<dvec2*>(y_);
    for (int j = k - 1; j >= 0; --j) {
        dvec2 t = gv[(size_t)j * L + c];
        for (int l = j + 1; l < k; ++l)
            t += cmul(R[((size_t)j * kMaxBasis + l) * L + c], y[(size_t)l * L + c]);  // y holds -y_l
        const dvec2 rjj = R[((size_t)j * kMaxBasis + j) * L + c];
        const double den = rjj.x * rjj.x + rjj.y * rjj.y;
        // -y_j = -(t / r_jj); a zero pivot only occurs for an all-zero column
        y[(size_t)j * L + c] = den > 0.0 ? cmulc(rjj, t) * (-1.0 / den) : dvec2{0.0, 0.0};
    }
}

__global__ __launch_bounds__(256)
void colnorm_kernel(const double* __restrict__ pn, int nch, int ldx, double* __restrict__ out) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ldx) return;
    double nn = 0.0;
    for (int ch = 0; ch < nch; ++ch) nn += pn[(size_t)ch * ldx + c];
    out[c] = sqrt(nn);
}

template <int KB>
hipError_t launch_gs_kb(int mode, const GsPass& p, dim3 grid, hipStream_t st) {
    switch (mode) {
        case GS_DOTS:
            hipLaunchKernelGGL((gs_kernel<KB, false, true, false, false>), grid, dim3(kGsThreads), 0,
                               st, p);
            break;
        case GS_PROJ_DOTS:
            hipLaunchKernelGGL((gs_kernel<KB, true, true, false, false>), grid, dim3(kGsThreads), 0,
                               st, p);
            break;
        case GS_UPDATE_NORM:
            hipLaunchKernelGGL((gs_kernel<KB, true, false, true, true>), grid, dim3(kGsThreads), 0,
                               st, p);
            break;
        case GS_UPDATE:
            hipLaunchKernelGGL((gs_kernel<KB, true, false, false, true>), grid, dim3(kGsThreads), 0,
                               st, p);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace

int gs_chunks(int rows, int ldx) {
    const int strips = (ldx + kGsCols - 1) / kGsCols;
    int nch = (16384 + strips - 1) / strips;
    const int cap = (rows + 63) / 64;
    if (nch > cap) nch = cap;
    if (nch > 64) nch = 64;
    return nch < 1 ? 1 : nch;
}

hipError_t launch_gs(int mode, const GsPass& p, hipStream_t st) {
    if (p.k < 0 || p.k > kMaxBasis || p.rows < 1 || p.ldx < 1 || p.chunk_rows < 1)
        return hipErrorInvalidValue;
    const dim3 grid((p.ldx + kGsCols - 1) / kGsCols, (p.rows + p.chunk_rows - 1) / p.chunk_rows);
    if (mode == GS_NORM) {
        hipLaunchKernelGGL((gs_kernel<1, false, false, true, false>), grid, dim3(kGsThreads), 0, st,
                           p);
        return hipGetLastError();
    }
    if (p.k < 1) return hipErrorInvalidValue;
    if (p.k <= 1) return launch_gs_kb<1>(mode, p, grid, st);
    if (p.k <= 2) return launch_gs_kb<2>(mode, p, grid, st);
    if (p.k <= 4) return launch_gs_kb<4>(mode, p, grid, st);
    if (p.k <= 8) return launch_gs_kb<8>(mode, p, grid, st);
    return launch_gs_kb<kMaxBasis>(mode, p, grid, st);
}

hipError_t launch_givens(const GivensArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(givens_kernel, dim3((a.ldx + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_gmres_solve(const double2* R, const double2* gv, double2* y, int k, int ldx,
                              hipStream_t st) {
    hipLaunchKernelGGL(gmres_solve_kernel, dim3((ldx + 255) / 256), dim3(256), 0, st, R, gv, y, k,
                       ldx);
    return hipGetLastError();
}

hipError_t launch_colnorm(const double* pn, int nch, int ldx, double* out, hipStream_t st) {
    hipLaunchKernelGGL(colnorm_kernel, dim3((ldx + 255) / 256), dim3(256), 0, st, pn, nch, ldx,
                       out);
    return hipGetLastError();
}

}  // namespace scd

// Memory-bound helper kernels of the Dyson solve: operand preparation, block
// initialisation, the convergence reduction, extraction of the kept blocks and
// the local observables (Sec. III.A of arXiv:1309.5994).
#include "internal.h"

namespace scd {
namespace {

// The GEMM's left operand, zero padded to mp x mp:
//   forward system     St[i][c][a] = S_i[a][c]   w_c J(z_c)   (S_i diag(wJ), transposed)
//   transposed system  St[i][c][a] = S_i[c][a]   w_c J(z_c)   (S_i^T diag(wJ), transposed)
// The contour weight and hopping of the summed-over time c are folded in once,
// so a sweep is X' = X0 + St^T (sum of neighbour tiles).  32x32 tiles go
// through LDS so both sides stay coalesced.
__global__ __launch_bounds__(256)
void scale_transpose_kernel(const double2* __restrict__ S, const double* __restrict__ J,
                            double2* __restrict__ St, int transposed_system, Geom g) {
    __shared__ double2 tile[32][33];
    const int site = blockIdx.z;
    const int a0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const double2* Si = S + (size_t)site * g.n_t * g.n_t;
    double2* Sti = St + (size_t)site * g.mp * g.mp;
    if (transposed_system) {
        // Row c of S_i scaled by wJ[c], stored as row c of St.
        for (int r = ty; r < 32; r += 8) {
            const int c = a0 + r, a = c0 + tx;
            if (c >= g.mp || a >= g.mp) continue;
            double2 v = make_double2(0.0, 0.0);
            if (c < g.n_t && a < g.n_t) {
                const double2 s = Si[(size_t)c * g.n_t + a];
                const double2 w = contour_wj(c, g.n_real, g.dt, g.dtau, J);
                v = make_double2(s.x * w.x - s.y * w.y, s.x * w.y + s.y * w.x);
            }
            Sti[(size_t)c * g.mp + a] = v;
        }
        return;
    }
    for (int r = ty; r < 32; r += 8) {
        const int a = a0 + r, c = c0 + tx;
        double2 v = make_double2(0.0, 0.0);
        if (a < g.n_t && c < g.n_t) {
            const double2 s = Si[(size_t)a * g.n_t + c];
            const double2 w = contour_wj(c, g.n_real, g.dt, g.dtau, J);
            v = make_double2(s.x * w.x - s.y * w.y, s.x * w.y + s.y * w.x);
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int c = c0 + r, a = a0 + tx;
        if (c < g.mp && a < g.mp) Sti[(size_t)c * g.mp + a] = tile[tx][r];
    }
}

// X = X0 = E_J S (the preconditioned unit-vector bundle of the block): zero
// except on each source's own site, which holds S_j[:, b] (whole sources),
// S_j[:, fixed] or S_j[fixed, :] (one column per source).  Xn, if given, is
// cleared.
__global__ __launch_bounds__(256)
void init_block_kernel(const double2* __restrict__ S, const int* __restrict__ src_blk, int bs,
                       int ldx, int x0_kind, int x0_fixed, double2* __restrict__ X,
                       double2* __restrict__ Xn, Geom g) {
    // One row (target site i, contour index a) at a time, its columns across
    // the threads (coalesced, 32-bit index arithmetic).
    const int cps = x0_kind == X0_BLOCK ? g.n_t : 1;
    const int rows = g.n_r * g.mp;
    for (int r = blockIdx.x; r < rows; r += gridDim.x) {
        const int i = r / g.mp, a = r - (r / g.mp) * g.mp;
        const double2* Si = S + (size_t)i * g.n_t * g.n_t;
        dvec2* Xr = reinterpret_cast<dvec2*>(X) + (size_t)r * ldx;
        dvec2* Xnr = Xn ? reinterpret_cast<dvec2*>(Xn) + (size_t)r * ldx : nullptr;
        for (int col = threadIdx.x; col < ldx; col += blockDim.x) {
            double2 v = make_double2(0.0, 0.0);
            const int s = col / cps;
            if (a < g.n_t && s < bs && src_blk[s] == i) {
                if (x0_kind == X0_COL_T)
                    v = Si[(size_t)x0_fixed * g.n_t + a];
                else if (x0_kind == X0_COL)
                    v = Si[(size_t)a * g.n_t + x0_fixed];
                else
                    v = Si[(size_t)a * g.n_t + (col - s * cps)];
            }
            __builtin_nontemporal_store(dvec2{v.x, v.y}, &Xr[col]);
            if (Xnr) __builtin_nontemporal_store(dvec2{0.0, 0.0}, &Xnr[col]);
        }
    }
}

// Order-independent max of the per-workgroup (|dX|max, |X|max, nan flag)
// partials into one slot; values are non-negative so their bit patterns order
// like unsigned integers.
__global__ __launch_bounds__(256)
void reduce_max3_kernel(const double* __restrict__ partial, int n,
                        unsigned long long* __restrict__ slot) {
    __shared__ double red[3][256];
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
        m0 = fmax(m0, partial[3 * k + 0]);
        m1 = fmax(m1, partial[3 * k + 1]);
        m2 = fmax(m2, partial[3 * k + 2]);
    }
    red[0][threadIdx.x] = m0;
    red[1][threadIdx.x] = m1;
    red[2][threadIdx.x] = m2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            for (int q = 0; q < 3; ++q)
                red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        for (int q = 0; q < 3; ++q)
            atomicMax(slot + q, (unsigned long long)__double_as_longlong(red[q][0]));
    }
}

// Copy the kept blocks of a converged column block out of the iterate.
__global__ __launch_bounds__(256)
void extract_kernel(const double2* __restrict__ X, int ldx, const int* __restrict__ src_blk,
                    int bs, int blk_start, int n_src, double2* __restrict__ G_cols,
                    double2* __restrict__ G_loc, double2* __restrict__ G_nn, Geom g) {
    const int n_t = g.n_t;
    const size_t blk_elems = (size_t)bs * n_t * n_t;
    // Part 1: local and neighbour blocks, (s, slot 0..4, a, b).
    const size_t kept = blk_elems * 5;
    const size_t cols_total = G_cols ? (size_t)g.n_r * n_t * bs * n_t : 0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < kept + cols_total;
         e += (size_t)gridDim.x * blockDim.x) {
        if (e < kept) {
            const int b = (int)(e % n_t);
            const int a = (int)((e / n_t) % n_t);
            const int q = (int)((e / ((size_t)n_t * n_t)) % 5);
            const int s = (int)(e / ((size_t)n_t * n_t * 5));
            const int j = src_blk[s];
            int k = j;
            if (q > 0) {
                int nb[4];
                site_neighbours(j, g.Lx, g.Ly, g.periodic, nb);
                k = nb[q - 1];
            }
            double2 v = make_double2(0.0, 0.0);
            if (k >= 0) v = X[((size_t)k * g.mp + a) * ldx + (size_t)s * n_t + b];
            const size_t gs = (size_t)(blk_start + s);
            if (q == 0) {
                G_loc[(gs * n_t + a) * n_t + b] = v;
            } else if (G_nn) {
                G_nn[((gs * 4 + (q - 1)) * n_t + a) * n_t + b] = v;
            }
        } else {
            const size_t f = e - kept;
            const int col = (int)(f % ((size_t)bs * n_t));
            const int a = (int)((f / ((size_t)bs * n_t)) % n_t);
            const int k = (int)(f / ((size_t)bs * n_t * n_t));
            G_cols[((size_t)k * n_t + a) * ((size_t)n_src * n_t) + (size_t)blk_start * n_t + col] =
                X[((size_t)k * g.mp + a) * ldx + col];
        }
    }
}

// n_s(t_a) = Im G_loc[s][a][b(a)]; ekin_s(t_a) = Re(-i J(t_a) sum_d G_nn[s][d][a][b(a)]),
// the expectation of the site's hopping terms for the +J hopping G is solved with.
__global__ __launch_bounds__(256)
void observables_kernel(const double2* __restrict__ G_loc, const double2* __restrict__ G_nn,
                        const double* __restrict__ J, int n_src, double* __restrict__ n_out,
                        double* __restrict__ ekin_out, Geom g) {
    const int n_t = g.n_t, n_real = g.n_real;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_src * n_real) return;
    const int s = e / n_real, a = e - (e / n_real) * n_real;
    const int b = 2 * n_real - 1 - a;
    n_out[e] = G_loc[((size_t)s * n_t + a) * n_t + b].y;
    if (ekin_out) {
        double im = 0.0;
        for (int d = 0; d < 4; ++d) im += G_nn[(((size_t)s * 4 + d) * n_t + a) * n_t + b].y;
        // Re(-i J (x + i y)) = J y
        ekin_out[e] = J[a] * im;
    }
}

// Double occupancy D_s(t_a) of source site j = src[s] from eq. docc:
//   U(t_a) D = Re dG - eps_j n_s(t_a) - ekin_s(t_a),
// dG the one-sided time derivative of G_loc at equal times (App. B), t' = t^+
// held at the backward point b(a):  (G[a][b] - G[a-1][b]) / dt for a >= 1,
// (G[1][b] - G[0][b]) / dt at a = 0; eps_j = V_j - U(t_min)/2 - mu.
__global__ __launch_bounds__(256)
void docc_kernel(const double2* __restrict__ G_loc, const double2* __restrict__ G_nn,
                 const double* __restrict__ J, const double* __restrict__ V,
                 const double* __restrict__ U, const int* __restrict__ src, int n_src,
                 double* __restrict__ d_out, Geom g) {
    const int n_t = g.n_t, n_real = g.n_real;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n_src * n_real) return;
    const int s = e / n_real, a = e - (e / n_real) * n_real;
    const int b = 2 * n_real - 1 - a;
    const int prev = a >= 1 ? a - 1 : 1;
    const double2* Gs = G_loc + (size_t)s * n_t * n_t;
    const double2 gab = Gs[(size_t)a * n_t + b];
    const double2 gpb = Gs[(size_t)prev * n_t + b];
    const double dG = (a >= 1 ? gab.x - gpb.x : gpb.x - gab.x) / g.dt;
    double im = 0.0;
    for (int d = 0; d < 4; ++d) im += G_nn[(((size_t)s * 4 + d) * n_t + a) * n_t + b].y;
    const double ekin = J[a] * im;
    const double eps = V[src[s]] - 0.5 * U[0] - g.mu;
    d_out[e] = (dG - eps * gab.y - ekin) / U[a];
}

// D~(t_a) = 2 sum_s D_s / (2 sum_s n_s): the doubly occupied fraction of the
// listed sites (one thread per time, sources summed in order).
__global__ __launch_bounds__(256)
void docc_fraction_kernel(const double2* __restrict__ G_loc, const double* __restrict__ d,
                          int n_src, double* __restrict__ frac, Geom g) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= g.n_real) return;
    const int n_t = g.n_t, b = 2 * g.n_real - 1 - a;
    double sd = 0.0, sn = 0.0;
    for (int s = 0; s < n_src; ++s) {
        sd += d[(size_t)s * g.n_real + a];
        sn += G_loc[((size_t)s * n_t + a) * n_t + b].y;
    }
    frac[a] = sd / sn;
}

// Elementwise helpers of mixed-precision refinement.
__global__ __launch_bounds__(256)
void to_f32_kernel(const dvec2* __restrict__ in, fvec2* __restrict__ out, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const dvec2 v = in[e];
        out[e] = fvec2{(float)v.x, (float)v.y};
    }
}

// X += D: the FP64 iterate absorbs the low-precision correction.  Each thread
// takes four elements a workgroup-width apart (every load and store of a wave
// is one contiguous run), all loads issued before the adds; nontemporal,
// since each byte is touched once.
__global__ __launch_bounds__(256)
void axpy_kernel(dvec2* __restrict__ X, const fvec2* __restrict__ D, size_t n) {
    const size_t span = 4 * (size_t)blockDim.x;
    for (size_t b = (size_t)blockIdx.x * span; b < n; b += (size_t)gridDim.x * span) {
        dvec2 x[4];
        fvec2 d[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t e = b + (size_t)k * blockDim.x + threadIdx.x;
            if (e < n) {
                x[k] = __builtin_nontemporal_load(&X[e]);
                d[k] = __builtin_nontemporal_load(&D[e]);
            }
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const size_t e = b + (size_t)k * blockDim.x + threadIdx.x;
            if (e < n)
                __builtin_nontemporal_store(x[k] + dvec2{(double)d[k].x, (double)d[k].y}, &X[e]);
        }
    }
}

}  // namespace

hipError_t launch_to_f32(const double2* in, void* out, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(to_f32_kernel, dim3(4096), dim3(256), 0, st,
                       reinterpret_cast<const dvec2*>(in), reinterpret_cast<fvec2*>(out), n);
    return hipGetLastError();
}

hipError_t launch_axpy_f32_to_f64(double2* X, const void* D32, size_t n, hipStream_t st) {
    hipLaunchKernelGGL(axpy_kernel, dim3(4096), dim3(256), 0, st, reinterpret_cast<dvec2*>(X),
                       reinterpret_cast<const fvec2*>(D32), n);
    return hipGetLastError();
}

hipError_t launch_scale_transpose(const Geom& g, const double2* S, const double* J, double2* St,
                                  int transposed_system, hipStream_t st) {
    dim3 grid((g.mp + 31) / 32, (g.mp + 31) / 32, g.n_r);
    hipLaunchKernelGGL(scale_transpose_kernel, grid, dim3(256), 0, st, S, J, St, transposed_system,
                       g);
    return hipGetLastError();
}

hipError_t launch_init_block(const Geom& g, const double2* S, const int* src_blk, int bs, int ldx,
                             int x0_kind, int x0_fixed, double2* X, double2* Xn, hipStream_t st) {
    hipLaunchKernelGGL(init_block_kernel, dim3(4096), dim3(256), 0, st, S, src_blk, bs, ldx, x0_kind,
                       x0_fixed, X, Xn, g);
    return hipGetLastError();
}

hipError_t launch_reduce_max3(const double* partial, int n, unsigned long long* slot,
                              hipStream_t st) {
    int blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(reduce_max3_kernel, dim3(blocks), dim3(256), 0, st, partial, n, slot);
    return hipGetLastError();
}

hipError_t launch_extract(const Geom& g, const double2* X, int ldx, const int* src_blk, int bs,
                          int blk_start, int n_src, double2* G_cols, double2* G_loc, double2* G_nn,
                          hipStream_t st) {
    hipLaunchKernelGGL(extract_kernel, dim3(4096), dim3(256), 0, st, X, ldx, src_blk, bs,
                       blk_start, n_src, G_cols, G_loc, G_nn, g);
    return hipGetLastError();
}

hipError_t launch_docc(const Geom& g, const double2* G_loc, const double2* G_nn, const double* J,
                       const double* V, const double* U, const int* src, int n_src, double* d_out,
                       double* frac_out, hipStream_t st) {
    const int total = n_src * g.n_real;
    hipLaunchKernelGGL(docc_kernel, dim3((total + 255) / 256), dim3(256), 0, st, G_loc, G_nn, J, V,
                       U, src, n_src, d_out, g);
    if (frac_out)
        hipLaunchKernelGGL(docc_fraction_kernel, dim3((g.n_real + 255) / 256), dim3(256), 0, st,
                           G_loc, d_out, n_src, frac_out, g);
    return hipGetLastError();
}

hipError_t launch_observables(const Geom& g, const double2* G_loc, const double2* G_nn,
                              const double* J, int n_src, double* n_out, double* ekin_out,
                              hipStream_t st) {
    const int total = n_src * g.n_real;
    hipLaunchKernelGGL(observables_kernel, dim3((total + 255) / 256), dim3(256), 0, st, G_loc,
                       G_nn, J, n_src, n_out, ekin_out, g);
    return hipGetLastError();
}

}  // namespace scd

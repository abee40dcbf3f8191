// Adjoint of the density loss L = sum_l w_l n_l(t_e), n_l(t_e) = Im G[(l,e),(l,b_e)]
// (b_e = 2 n_real - 1 - e, the backward partner of forward point e).
//
// With G = (I - S D)^-1 S, (I - S D)^-1 = I + G D and D symmetric:
//   g_l = G v_l            one forward column per site (v_l: unit vector at (l, b_e))
//   h_l = G^T u_l          one column of the transposed system (u_l: unit vector at (l, e)),
//                          G^T = (I - S^T D)^-1 S^T, so h solves the same kind of Dyson
//                          equation with every S_i transposed
//   dL = Im sum_j <Lam_j, dS_j> + Im sum_c (dL/dJ_c) dJ_c
//   Lam_j[a][b] = sum_l w_l P_j[a][l] Q_j[b][l],
//   P_j[a][l] = delta_jl delta_ae   + wJ_a sum_{k in nbr(j)} h_l[(k,a)]     (u + D h)
//   Q_j[b][l] = delta_jl delta_bbe  + wJ_b sum_{k in nbr(j)} g_l[(k,b)]     (v + D g)
//   dL/dJ_c  = Im w_c sum_l w_l sum_i h_l[(i,c)] sum_{k in nbr(i)} g_l[(k,c)]
// The per-site derivatives dS_j/d eps_j and dS_j/dU_k are the closed form of
// the atomic Green's function (Sec. III of arXiv:1309.5994) differentiated:
// each of its two terms T_nu = (-/+ i) exp(log p_nu + d) contributes
// T_nu (d log p_nu / dx + d d / dx).
//
// The g and h columns come from the sweep kernels (one column per source
// site, X0_COL / X0_COL_T); this file holds the kernels that turn them into
// gradients.  Iterates are [N_r][mp][ldx] complex128 with column l = source l.
#include "internal.h"

namespace scd {
namespace {

struct AdjArgs {
    int ldx;        // padded column count of the one-column-per-site iterates
    int e, be;      // forward loss point and its backward partner
};

__device__ inline dvec2 cmul(dvec2 a, dvec2 b) {
    return dvec2{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Sum of the neighbour rows of an iterate: sum_{k in nbr(i)} X[k][a][l].
__device__ inline dvec2 nbr_sum(const dvec2* X, const int nb[4], int a, int l, int mp, int ldx) {
    dvec2 s = dvec2{0.0, 0.0};
#pragma unroll
    for (int d = 0; d < 4; ++d)
        if (nb[d] >= 0) s += X[((size_t)nb[d] * mp + a) * ldx + l];
    return s;
}

// Lam_j for one site and one 32x32 (a, b) tile, reduced over all l in chunks of
// 32 staged through LDS (P and Q formed on the fly from the h and g iterates).
constexpr int kLT = 32;
__global__ __launch_bounds__(256)
void lambda_kernel(const dvec2* __restrict__ H, const dvec2* __restrict__ Gc,
                   const double* __restrict__ J, const double* __restrict__ w,
                   dvec2* __restrict__ Lam, Geom g, AdjArgs aa) {
    __shared__ dvec2 Ps[kLT][kLT + 1];   // [a][l]
    __shared__ dvec2 Qs[kLT][kLT + 1];   // [b][l]  (already multiplied by w_l)
    const int j = blockIdx.z;
    const int a0 = blockIdx.y * kLT, b0 = blockIdx.x * kLT;
    const int tid = threadIdx.x;
    const int tr = tid / 16, tc = tid % 16;     // each thread: rows a0+tr, a0+tr+16; cols b0+tc, b0+tc+16
    int nb[4];
    site_neighbours(j, g.Lx, g.Ly, g.periodic, nb);
    dvec2 acc[2][2];
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) acc[p][q] = dvec2{0.0, 0.0};
    for (int l0 = 0; l0 < g.n_r; l0 += kLT) {
        for (int e = tid; e < kLT * kLT; e += 256) {
            const int r = e / kLT, l = l0 + e % kLT;
            dvec2 pv = dvec2{0.0, 0.0}, qv = dvec2{0.0, 0.0};
            const int a = a0 + r, b = b0 + r;
            if (l < g.n_r) {
                if (a < g.n_t) {
                    const double2 wj = contour_wj(a, g.n_real, g.dt, g.dtau, J);
                    pv = cmul(dvec2{wj.x, wj.y}, nbr_sum(H, nb, a, l, g.mp, aa.ldx));
                    if (l == j && a == aa.e) pv.x += 1.0;
                }
                if (b < g.n_t) {
                    const double2 wj = contour_wj(b, g.n_real, g.dt, g.dtau, J);
                    qv = cmul(dvec2{wj.x, wj.y}, nbr_sum(Gc, nb, b, l, g.mp, aa.ldx));
                    if (l == j && b == aa.be) qv.x += 1.0;
                    qv *= w[l];
                }
            }
            Ps[r][e % kLT] = pv;
            Qs[r][e % kLT] = qv;
        }
        __syncthreads();
#pragma unroll 4
        for (int l = 0; l < kLT; ++l) {
            const dvec2 p0 = Ps[tr][l], p1 = Ps[tr + 16][l];
            const dvec2 q0 = Qs[tc][l], q1 = Qs[tc + 16][l];
            acc[0][0] += cmul(p0, q0);
            acc[0][1] += cmul(p0, q1);
            acc[1][0] += cmul(p1, q0);
            acc[1][1] += cmul(p1, q1);
        }
        __syncthreads();
    }
    for (int p = 0; p < 2; ++p)
        for (int q = 0; q < 2; ++q) {
            const int a = a0 + tr + 16 * p, b = b0 + tc + 16 * q;
            if (a < g.n_t && b < g.n_t) Lam[((size_t)j * g.n_t + a) * g.n_t + b] = acc[p][q];
        }
}

// Per-site contraction of Lam_j with the closed-form derivatives of S_j.
// Outputs: dV[j] = Im <Lam_j, dS_j/deps>, bz[j] = Im <Lam_j, dS_j/dU0 (Boltzmann part)>,
// and the row / column sums r_j[a] = sum_b Lam t2, c_j[b] = sum_a Lam t2 of the
// second term t2, from which the phase-integral part of dL/dU_k follows.
__global__ __launch_bounds__(256)
void contract_kernel(const dvec2* __restrict__ Lam, const double* __restrict__ V,
                     const double* __restrict__ U, double* __restrict__ dV,
                     double* __restrict__ bz, dvec2* __restrict__ rsum, dvec2* __restrict__ csum,
                     Geom g) {
    __shared__ double z_re[1024], z_im[1024], ph_re[1024], ph_im[1024], cum[512];
    __shared__ double red[2][256];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    const int n_t = g.n_t, n_real = g.n_real;
    if (tid == 0) {
        double acc = 0.0;
        cum[0] = 0.0;
        for (int k = 1; k < n_real; ++k) {
            acc += 0.5 * (U[k] + U[k - 1]) * g.dt;
            cum[k] = acc;
        }
    }
    __syncthreads();
    for (int a = tid; a < n_t; a += 256) {
        if (a < 2 * n_real) {
            const int k = a < n_real ? a : 2 * n_real - 1 - a;
            z_re[a] = k * g.dt;
            z_im[a] = 0.0;
            ph_re[a] = cum[k];
            ph_im[a] = 0.0;
        } else {
            const double tau = (a - 2 * n_real + 1) * g.dtau;
            z_re[a] = 0.0;
            z_im[a] = -tau;
            ph_re[a] = 0.0;
            ph_im[a] = -tau * U[0];
        }
    }
    __syncthreads();
    const double U0 = U[0];
    const double eps = V[j] - 0.5 * U0 - g.mu;
    const double lw1 = -g.beta * eps, lw3 = -g.beta * (2.0 * eps + U0);
    const double mx = fmax(fmax(0.0, lw1), lw3);
    const double lz = mx + log(exp(-mx) + 2.0 * exp(lw1 - mx) + exp(lw3 - mx));
    const double lp[4] = {-lz, lw1 - lz, lw1 - lz, lw3 - lz};
    const double p1 = exp(lp[1]), p3 = exp(lp[3]);
    const double meanN = 2.0 * p1 + 2.0 * p3;     // <N> = p1 + p2 + 2 p3, p1 = p2
    const double dlde[4] = {-g.beta * (0.0 - meanN), -g.beta * (1.0 - meanN),
                            -g.beta * (1.0 - meanN), -g.beta * (2.0 - meanN)};
    const double dldu[4] = {g.beta * p3, g.beta * p3, g.beta * p3, -g.beta * (1.0 - p3)};
    const dvec2* Lj = Lam + (size_t)j * n_t * n_t;

    // Term pair of S[a][b]: returns t1, t2 (complex) and the indices of their weights.
    auto terms = [&](int a, int b, dvec2& t1, dvec2& t2, int& n1, int& n2) {
        const double dzr = z_re[a] - z_re[b], dzi = z_im[a] - z_im[b];
        const double d1r = eps * dzi, d1i = -eps * dzr;
        const double d2r = d1r + (ph_im[a] - ph_im[b]);
        const double d2i = d1i - (ph_re[a] - ph_re[b]);
        const bool greater = a > b;
        n1 = greater ? 0 : 2;
        n2 = greater ? 1 : 3;
        double s1, c1, s2, c2;
        sincos(d1i, &s1, &c1);
        sincos(d2i, &s2, &c2);
        const double m1 = exp(lp[n1] + d1r), m2 = exp(lp[n2] + d2r);
        // greater: -i (m e^{i d}) ; lesser: +i (m e^{i d})
        const double sg = greater ? -1.0 : 1.0;
        t1 = dvec2{-sg * m1 * s1, sg * m1 * c1};
        t2 = dvec2{-sg * m2 * s2, sg * m2 * c2};
    };

    double de = 0.0, db = 0.0;
    for (int a = tid; a < n_t; a += 256) {
        dvec2 racc = dvec2{0.0, 0.0};
        for (int b = 0; b < n_t; ++b) {
            dvec2 t1, t2;
            int n1, n2;
            terms(a, b, t1, t2, n1, n2);
            const dvec2 L = Lj[(size_t)a * n_t + b];
            // d(-i(z_a - z_b)) / d eps = -i dz  ->  (dzi, -dzr)
            const dvec2 ddz = dvec2{z_im[a] - z_im[b], -(z_re[a] - z_re[b])};
            const dvec2 dS = (t1 * dlde[n1] + cmul(t1, ddz)) + (t2 * dlde[n2] + cmul(t2, ddz));
            de += cmul(L, dS).y;
            db += cmul(L, t1 * dldu[n1] + t2 * dldu[n2]).y;
            racc += cmul(L, t2);
        }
        rsum[(size_t)j * n_t + a] = racc;
    }
    for (int b = tid; b < n_t; b += 256) {
        dvec2 cacc = dvec2{0.0, 0.0};
        for (int a = 0; a < n_t; ++a) {
            dvec2 t1, t2;
            int n1, n2;
            terms(a, b, t1, t2, n1, n2);
            cacc += cmul(Lj[(size_t)a * n_t + b], t2);
        }
        csum[(size_t)j * n_t + b] = cacc;
    }
    red[0][tid] = de;
    red[1][tid] = db;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    if (tid == 0) {
        dV[j] = red[0][0];
        bz[j] = red[1][0];
    }
}

// dL/dU_k = Im(-i sum_a jac[a][k] (R[a] - C[a])) + [k = 0] (sum_j bz_j - 1/2 sum_j dV_j),
// R = sum_j r_j, C = sum_j c_j, jac[a][k] = d Phi_U(z_a) / dU_k of the trapezoid phase.
__global__ __launch_bounds__(256)
void finalize_u_kernel(const dvec2* __restrict__ rsum, const dvec2* __restrict__ csum,
                       const double* __restrict__ dV, const double* __restrict__ bz,
                       double* __restrict__ dU, Geom g) {
    __shared__ dvec2 RC[1024];
    __shared__ double red[2][256];
    const int tid = threadIdx.x;
    const int n_t = g.n_t, n_real = g.n_real;
    for (int a = tid; a < n_t; a += 256) {
        dvec2 s = dvec2{0.0, 0.0};
        for (int j = 0; j < g.n_r; ++j) s += rsum[(size_t)j * n_t + a] - csum[(size_t)j * n_t + a];
        RC[a] = s;
    }
    double sv = 0.0, sb = 0.0;
    for (int j = tid; j < g.n_r; j += 256) {
        sv += dV[j];
        sb += bz[j];
    }
    red[0][tid] = sv;
    red[1][tid] = sb;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) {
            red[0][tid] += red[0][tid + w];
            red[1][tid] += red[1][tid + w];
        }
        __syncthreads();
    }
    for (int k = tid; k < n_real; k += 256) {
        // sum_a jac[a][k] RC[a]: real points with forward index m >= 1 carry dt/2 at
        // k = 0 and k = m, dt for 0 < k < m; imaginary points carry (z_a - t_min) at k = 0.
        dvec2 s = dvec2{0.0, 0.0};
        for (int a = 0; a < 2 * n_real; ++a) {
            const int m = a < n_real ? a : 2 * n_real - 1 - a;
            if (m == 0 || k > m) continue;
            const double wgt = (k == 0 || k == m) ? 0.5 * g.dt : g.dt;
            s += RC[a] * wgt;
        }
        if (k == 0) {
            for (int a = 2 * n_real; a < n_t; ++a) {
                const double tau = (a - 2 * n_real + 1) * g.dtau;   // jac = -i tau
                s += dvec2{RC[a].y * tau, -RC[a].x * tau};
            }
        }
        // Im(-i s) = -Re(s)
        double v = -s.x;
        if (k == 0) v += red[1][0] - 0.5 * red[0][0];
        dU[k] = v;
    }
}

// dL/dJ_c per contour point, then summed onto the physical times.
__global__ __launch_bounds__(256)
void dj_kernel(const dvec2* __restrict__ H, const dvec2* __restrict__ Gc,
               const double* __restrict__ w, double* __restrict__ djc, Geom g, AdjArgs aa) {
    __shared__ double red[256];
    const int c = blockIdx.x;
    const int tid = threadIdx.x;
    dvec2 acc = dvec2{0.0, 0.0};
    const size_t pairs = (size_t)g.n_r * g.n_r;
    for (size_t e = tid; e < pairs; e += 256) {
        const int i = (int)(e / g.n_r), l = (int)(e % g.n_r);
        int nb[4];
        site_neighbours(i, g.Lx, g.Ly, g.periodic, nb);
        const dvec2 hv = H[((size_t)i * g.mp + c) * aa.ldx + l];
        acc += cmul(hv, nbr_sum(Gc, nb, c, l, g.mp, aa.ldx)) * w[l];
    }
    // Im(w_c acc): w_c = dt, -dt or -i dtau
    double v;
    if (c < g.n_real) v = g.dt * acc.y;
    else if (c < 2 * g.n_real) v = -g.dt * acc.y;
    else v = -g.dtau * acc.x;
    red[tid] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s) red[tid] += red[tid + s];
        __syncthreads();
    }
    if (tid == 0) djc[c] = red[0];
}

__global__ __launch_bounds__(256)
void finalize_j_kernel(const double* __restrict__ djc, double* __restrict__ dJ, Geom g) {
    for (int k = threadIdx.x; k < g.n_real; k += 256) {
        double v = djc[k] + djc[2 * g.n_real - 1 - k];
        if (k == 0)
            for (int c = 2 * g.n_real; c < g.n_t; ++c) v += djc[c];
        dJ[k] = v;
    }
}

// n_l(t_e) = Im g_l[(l, e)] for every site, and L = sum_l w_l n_l(t_e).
__global__ __launch_bounds__(256)
void loss_kernel(const dvec2* __restrict__ Gc, const double* __restrict__ w,
                 double* __restrict__ n_te, double* __restrict__ loss, Geom g, AdjArgs aa) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int l = threadIdx.x; l < g.n_r; l += 256) {
        const double v = Gc[((size_t)l * g.mp + aa.e) * aa.ldx + l].y;
        if (n_te) n_te[l] = v;
        if (w) acc += w[l] * v;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && loss) *loss = red[0];
}

}  // namespace

hipError_t launch_adjoint_grads(const Geom& g, int ldx, int e, const double2* H, const double2* Gc,
                                const double* V, const double* U, const double* J, const double* w,
                                double2* Lam, double2* rsum, double2* csum, double* bz, double* djc,
                                double* dV, double* dU, double* dJ, hipStream_t st) {
    AdjArgs aa{ldx, e, 2 * g.n_real - 1 - e};
    const dvec2* H_ = reinterpret_cast<const dvec2*>(H);
    const dvec2* G_ = reinterpret_cast<const dvec2*>(Gc);
    dim3 lg((g.n_t + kLT - 1) / kLT, (g.n_t + kLT - 1) / kLT, g.n_r);
    hipLaunchKernelGGL(lambda_kernel, lg, dim3(256), 0, st, H_, G_, J, w,
                       reinterpret_cast<dvec2*>(Lam), g, aa);
    hipLaunchKernelGGL(contract_kernel, dim3(g.n_r), dim3(256), 0, st,
                       reinterpret_cast<const dvec2*>(Lam), V, U, dV, bz,
                       reinterpret_cast<dvec2*>(rsum), reinterpret_cast<dvec2*>(csum), g);
    hipLaunchKernelGGL(finalize_u_kernel, dim3(1), dim3(256), 0, st,
                       reinterpret_cast<const dvec2*>(rsum), reinterpret_cast<const dvec2*>(csum),
                       dV, bz, dU, g);
    hipLaunchKernelGGL(dj_kernel, dim3(g.n_t), dim3(256), 0, st, H_, G_, w, djc, g, aa);
    hipLaunchKernelGGL(finalize_j_kernel, dim3(1), dim3(256), 0, st, djc, dJ, g);
    return hipGetLastError();
}

hipError_t launch_adjoint_loss(const Geom& g, int ldx, int e, const double2* Gc, const double* w,
                               double* n_te, double* loss, hipStream_t st) {
    AdjArgs aa{ldx, e, 2 * g.n_real - 1 - e};
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, reinterpret_cast<const dvec2*>(Gc), w,
                       n_te, loss, g, aa);
    return hipGetLastError();
}

}  // namespace scd

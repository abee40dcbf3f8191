// Atomic-limit contour Green's function of every lattice site (Sec. III of
// arXiv:1309.5994): the closed form obtained by inserting the local time
// evolution (eq. localtimeevolution) between the number states, i.e. products
// of the tabulated phases zeta_nu of eq. cumulanttabulation.
//
// One workgroup per (site, slab of 1024 matrix elements).  Each workgroup
// first tabulates, in LDS, the complex contour time elapsed since t_min and the
// phase integral of U along the contour (trapezoid on the forward grid;
// backward points share their forward partner's value; imaginary points use
// U(t_min) times the elapsed imaginary time), then writes its elements with
// the Boltzmann weights combined in log space so that imaginary-branch factors
// exp(E tau) never overflow.
#include "internal.h"

namespace scd {
namespace {

constexpr int kSigmaThreads = 256;
constexpr int kSigmaPerThread = 4;

__global__ __launch_bounds__(kSigmaThreads)
void sigma_build_kernel(const double* __restrict__ V, const double* __restrict__ U,
                        double2* __restrict__ S, Geom g) {
    __shared__ double z_re[1024], z_im[1024];   // z_a - t_min
    __shared__ double ph_re[1024], ph_im[1024]; // int_{t_min}^{z_a} U dz
    __shared__ double cum[512];                 // trapezoid prefix of U on the forward grid

    const int n_t = g.n_t, n_real = g.n_real;
    const int site = blockIdx.y;
    const int tid = threadIdx.x;

    if (tid == 0) {
        double acc = 0.0;
        cum[0] = 0.0;
        for (int k = 1; k < n_real; ++k) {
            acc += 0.5 * (U[k] + U[k - 1]) * g.dt;
            cum[k] = acc;
        }
    }
    __syncthreads();
    for (int a = tid; a < n_t; a += kSigmaThreads) {
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

    // Level and log Boltzmann weights of the four number states at t_min.
    const double U0 = U[0];
    const double eps = V[site] - 0.5 * U0 - g.mu;
    const double lw1 = -g.beta * eps;
    const double lw3 = -g.beta * (2.0 * eps + U0);
    const double mx = fmax(fmax(0.0, lw1), lw3);
    const double lz = mx + log(exp(-mx) + 2.0 * exp(lw1 - mx) + exp(lw3 - mx));
    const double lp0 = -lz, lp1 = lw1 - lz, lp2 = lw1 - lz, lp3 = lw3 - lz;

    double2* Si = S + (size_t)site * n_t * n_t;
    const int total = n_t * n_t;
    const int base = blockIdx.x * (kSigmaThreads * kSigmaPerThread);
    for (int r = 0; r < kSigmaPerThread; ++r) {
        const int e = base + r * kSigmaThreads + tid;
        if (e >= total) break;
        const int a = e / n_t, b = e - (e / n_t) * n_t;
        // d1 = -i eps (z_a - z_b);  d2 = d1 - i (Phi_a - Phi_b)
        const double dzr = z_re[a] - z_re[b], dzi = z_im[a] - z_im[b];
        const double d1r = eps * dzi, d1i = -eps * dzr;
        const double d2r = d1r + (ph_im[a] - ph_im[b]);
        const double d2i = d1i - (ph_re[a] - ph_re[b]);
        const bool greater = a > b;
        const double l1 = greater ? lp0 : lp2;
        const double l2 = greater ? lp1 : lp3;
        double s1, c1, s2, c2;
        sincos(d1i, &s1, &c1);
        sincos(d2i, &s2, &c2);
        const double m1 = exp(l1 + d1r), m2 = exp(l2 + d2r);
        const double tr = m1 * c1 + m2 * c2;   // sum of the two terms, real part
        const double ti = m1 * s1 + m2 * s2;   // imaginary part
        // greater: -i (tr + i ti) = ti - i tr ; lesser: +i (tr + i ti) = -ti + i tr
        Si[e] = greater ? make_double2(ti, -tr) : make_double2(-ti, tr);
    }
}

}  // namespace

hipError_t launch_sigma_build(const Geom& g, const double* V, const double* U, double2* S,
                              hipStream_t st) {
    const int per_wg = kSigmaThreads * kSigmaPerThread;
    dim3 grid((g.n_t * g.n_t + per_wg - 1) / per_wg, g.n_r);
    hipLaunchKernelGGL(sigma_build_kernel, grid, dim3(kSigmaThreads), 0, st, V, U, S, g);
    return hipGetLastError();
}

}  // namespace scd

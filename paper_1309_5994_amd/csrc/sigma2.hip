// Second-order strong-coupling self-energy (Sec. III of arXiv:1309.5994,
// eq. defnSigmatilde, eq. defnSigma) and the dressed block diagonal it gives.
//
//   Sigma~_i(a, b) = - sum_{s1} sum_{c,d} G~_{up s1}(a, d; c, b) K_i(c, d),
//   K_i(c, d)      = w_c J(z_c) [sum_{k in nbr(i)} G_loc,k(c, d)] J(z_d) w_d,
//
// with the cumulant G~ = G^II + G(a,c) G(d,b) delta_{up s1} - G(a,b) G(d,c)
// (G = S_i, the atomic Green's function).  The one-particle terms of the
// cumulant collapse to matrix algebra,
//
//   Sigma~ = - sum_{c,d} K(c,d) [G^II_{up up} + G^II_{up dn}](a, d; c, b)
//            + 2 S(a,b) sum_{c,d} K(c,d) S(d,c) - sum_{c,d} S(a,c) K(c,d) S(d,b),
//
// so only the two-particle part is a sum over (c, d).  G^II is evaluated in
// the number basis |0>, |dn>, |up>, |up dn> (eq. cumulanttabulation): the four
// operators c_up(a) c_s1(d) c^dag_s1(c) c^dag_up(b) are put in contour order
// (later first; at one contour index creation operators count as later,
// operators of one kind keep their written order) with the permutation's sign,
// and every initial state is carried through the ordered product, each
// operator contributing exp(i Theta_after(z) - i Theta_before(z)); the phases
// and the Boltzmann weight are combined in one exponent, so imaginary-branch
// factors never overflow.  Each path is a product of single-time factors and
// the order changes with d only at d = a, b, c, so the d-sum is a difference
// of prefix sums and the contraction costs O(N_t^3) per site.
//
// The dressed block (the contour inverse of calG^-1 - Sigma, with
// Sigma = calG^-1 o Sigma~ o calG^-1) is S' = S (S - Sigma~)^-1 S in plain
// matrices; the lattice solve with S' in place of S is eq. Glatt with Sigma.
#include <algorithm>
#include <cstring>

#include "internal.h"

namespace scd {
namespace {

constexpr int kS2Threads = 256;
constexpr int kDressThreads = 1024;   // one workgroup per site: 16 waves to hide memory latency

__device__ inline double2 cmul2(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Transitions of the four operators c_up, c_dn, c^dag_up, c^dag_dn on the
// states 0 |0>, 1 |dn>, 2 |up>, 3 |up dn> = c^dag_up c^dag_dn |0>:
// next state (-1: annihilated) and sign.
constexpr int kNext[4][4] = {{-1, -1, 0, 1}, {-1, 0, -1, 2}, {2, 3, -1, -1}, {1, -1, 3, -1}};
constexpr int kAmp[4][4] = {{0, 0, 1, 1}, {0, 1, 0, -1}, {1, 1, 0, 0}, {1, 0, -1, 0}};

// The contour order of the four operators c_up(a), c_s1(d), c^dag_s1(c),
// c^dag_up(b) (written slots 0..3) is one of 24 permutations, fixed by the six
// pairwise key comparisons; for each permutation and neighbour spin the
// number-state paths that survive the ordered product are fixed too.  Per
// path: the initial state, the amplitude (transition signs times the
// permutation's sign) and, per written slot, which phase table its operator
// uses (0: e^{i T1}, 1: e^{-i T1}, 2: e^{i (T3 - T1)}, 3: e^{-i (T3 - T1)}).
struct PathTable {
    signed char perm_of[64];          // comparison bits -> permutation
    signed char npath[24][2];
    signed char nu[24][2][4];
    signed char amp[24][2][4];
    signed char tab[24][2][4][4];     // [perm][spin][path][written slot]
};

PathTable build_path_table() {
    PathTable T;
    std::memset(&T, 0, sizeof T);
    std::memset(T.perm_of, -1, sizeof T.perm_of);
    int order[4] = {0, 1, 2, 3};
    int p = 0;
    do {
        int rank[4];
        for (int q = 0; q < 4; ++q) rank[order[q]] = q;
        // bit for written pair (i, j), i < j: j precedes i in contour order
        const int pairs[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        int code = 0, inv = 0;
        for (int k = 0; k < 6; ++k) {
            const int i = pairs[k][0], j = pairs[k][1];
            if (rank[j] < rank[i]) {
                code |= 1 << k;
                ++inv;
            }
        }
        T.perm_of[code] = (signed char)p;
        const int sign = (inv & 1) ? -1 : 1;
        for (int s1 = 0; s1 < 2; ++s1) {
            const int kind_of[4] = {0, s1 == 0 ? 0 : 1, s1 == 0 ? 2 : 3, 2};
            int n = 0;
            for (int nu = 0; nu < 4; ++nu) {
                int st = nu, amp = sign;
                int tabs[4] = {0, 0, 0, 0};
                bool ok = true;
                for (int q = 3; q >= 0; --q) {          // rightmost operator acts first
                    const int slot = order[q];
                    const int kind = kind_of[slot];
                    const int nx = kNext[kind][st];
                    if (nx < 0) {
                        ok = false;
                        break;
                    }
                    amp *= kAmp[kind][st];
                    const bool creation = kind >= 2;
                    const bool two = st == 3 || nx == 3;
                    tabs[slot] = (two ? 2 : 0) + (creation ? 0 : 1);
                    st = nx;
                }
                if (!ok || st != nu) continue;
                T.nu[p][s1][n] = (signed char)nu;
                T.amp[p][s1][n] = (signed char)amp;
                for (int w = 0; w < 4; ++w) T.tab[p][s1][n][w] = (signed char)tabs[w];
                ++n;
            }
            T.npath[p][s1] = (signed char)n;
        }
        ++p;
    } while (std::next_permutation(order, order + 4));
    return T;
}

// K_i = diag(wJ) (sum of the neighbours' G_loc) diag(wJ), one thread per element.
__global__ __launch_bounds__(256)
void k_build_kernel(const double2* __restrict__ G_loc, const double* __restrict__ J,
                    double2* __restrict__ K, Geom g) {
    const int n_t = g.n_t;
    const size_t per = (size_t)n_t * n_t;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < (size_t)g.n_r * per;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / per);
        const int cd = (int)(e - (size_t)i * per);
        const int c = cd / n_t, d = cd - (cd / n_t) * n_t;
        int nb[4];
        site_neighbours(i, g.Lx, g.Ly, g.periodic, nb);
        double2 s = make_double2(0.0, 0.0);
        for (int q = 0; q < 4; ++q)
            if (nb[q] >= 0) {
                const double2 v = G_loc[(size_t)nb[q] * per + cd];
                s.x += v.x;
                s.y += v.y;
            }
        const double2 wc = contour_wj(c, g.n_real, g.dt, g.dtau, J);
        const double2 wd = contour_wj(d, g.n_real, g.dt, g.dtau, J);
        K[e] = cmul2(cmul2(wc, s), wd);
    }
}

// Contour phases of the site (LDS): Theta_1 = eps (z - t_min) (states |dn>,
// |up>) and Theta_3 = 2 eps (z - t_min) + int U dz (state |up dn>).
__device__ void site_phases(const double* U, double eps, Geom g, double* t1r, double* t1i,
                            double* t3r, double* t3i, double* cum) {
    const int n_t = g.n_t, n_real = g.n_real;
    if (threadIdx.x == 0) {
        double acc = 0.0;
        cum[0] = 0.0;
        for (int k = 1; k < n_real; ++k) {
            acc += 0.5 * (U[k] + U[k - 1]) * g.dt;
            cum[k] = acc;
        }
    }
    __syncthreads();
    for (int a = threadIdx.x; a < n_t; a += blockDim.x) {
        double zr, zi, pr, pi;
        if (a < 2 * n_real) {
            const int k = a < n_real ? a : 2 * n_real - 1 - a;
            zr = k * g.dt;
            zi = 0.0;
            pr = cum[k];
            pi = 0.0;
        } else {
            const double tau = (a - 2 * n_real + 1) * g.dtau;
            zr = 0.0;
            zi = -tau;
            pr = 0.0;
            pi = -tau * U[0];
        }
        t1r[a] = eps * zr;
        t1i[a] = eps * zi;
        t3r[a] = 2.0 * eps * zr + pr;
        t3i[a] = 2.0 * eps * zi + pi;
    }
    __syncthreads();
}

// part(a, b) = - sum_{c,d} K(c,d) [G^II_{up up} + G^II_{up dn}](a, d; c, b):
// one thread per (a, b), one workgroup per (site, 256 outputs).  The phase
// factor an operator at z contributes, exp(i (Theta_after - Theta_before)(z)),
// is one of four tabulated values (Theta_dn = Theta_up): e^{+-i Theta_1} for
// 0 <-> 1 particle, e^{+-i (Theta_3 - Theta_1)} for 1 <-> 2 particles.  Six
// key comparisons give the contour order's permutation, whose surviving
// number-state paths come from the path table (LDS).  Only three of the
// comparisons involve d, so per contour index c the workgroup stages the
// prefix sums over d of K(c, d) times the d factors, and each output applies
// the paths once per stretch of constant order (at most four per (a, b, c)).
// The tables are finite on the
// imaginary branch (|eps|, |eps + U| times beta stay far from the double
// range); the Boltzmann weight multiplies the product.
__global__ __launch_bounds__(kS2Threads)
void sigma2_pair_kernel(const double2* __restrict__ K, const double* __restrict__ V,
                        const double* __restrict__ U, double2* __restrict__ out, Geom g,
                        PathTable paths) {
    __shared__ double t1r[kMaxNt], t1i[kMaxNt], t3r[kMaxNt], t3i[kMaxNt];
    __shared__ double cum[kMaxNt];
    __shared__ double2 fac[4][kMaxNt];   // [0] e^{i T1}, [1] e^{-i T1}, [2] e^{i(T3-T1)}, [3] e^{-i(T3-T1)}
    __shared__ PathTable tb;
    // Prefix sums over d of row c: pz[0] + i pz[1] = sum_{d' < d} K(c, d')
    // e^{-i T1}(d'), pz[2] + i pz[3] the same with e^{-i (T3 - T1)}(d');
    // pz[.][0] = 0.
    __shared__ double pz[4][kMaxNt + 1];
    {
        const signed char* src = reinterpret_cast<const signed char*>(&paths);
        signed char* dst = reinterpret_cast<signed char*>(&tb);
        for (int k = threadIdx.x; k < (int)sizeof(PathTable); k += kS2Threads) dst[k] = src[k];
    }
    const int site = blockIdx.y;
    const int n_t = g.n_t;
    const double U0 = U[0];
    const double eps = V[site] - 0.5 * U0 - g.mu;
    site_phases(U, eps, g, t1r, t1i, t3r, t3i, cum);
    for (int z = threadIdx.x; z < n_t; z += kS2Threads) {
        // exp(i (x + i y)) = e^{-y} (cos x + i sin x)
        double s, c;
        sincos(t1r[z], &s, &c);
        double m = exp(-t1i[z]);
        fac[0][z] = make_double2(m * c, m * s);
        m = exp(t1i[z]);
        fac[1][z] = make_double2(m * c, -m * s);
        const double dr = t3r[z] - t1r[z], di = t3i[z] - t1i[z];
        sincos(dr, &s, &c);
        m = exp(-di);
        fac[2][z] = make_double2(m * c, m * s);
        m = exp(di);
        fac[3][z] = make_double2(m * c, -m * s);
    }
    __syncthreads();
    // Boltzmann weights of the four states at t_min
    const double lw1 = -g.beta * eps, lw3 = -g.beta * (2.0 * eps + U0);
    const double mx = fmax(fmax(0.0, lw1), lw3);
    const double lz = mx + log(exp(-mx) + 2.0 * exp(lw1 - mx) + exp(lw3 - mx));
    const double pw[4] = {exp(-lz), exp(lw1 - lz), exp(lw1 - lz), exp(lw3 - lz)};

    // Every thread takes part in staging the rows (barriers below); threads
    // past the last output only stage.
    static_assert(kS2Threads == 4 * 64, "one wave per scanned array");
    static_assert(kMaxNt <= kS2Threads, "one row element per thread");
    const int e = blockIdx.x * kS2Threads + threadIdx.x;
    const bool live = e < n_t * n_t;
    const int ec = live ? e : 0;
    const int a = ec / n_t, b = ec - (ec / n_t) * n_t;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double2* Ki = K + (size_t)site * n_t * n_t;
    double acc_r = 0.0, acc_i = 0.0;
    // Surviving paths of contour order `code`, with the d-sums P1 = sum K(c, d)
    // e^{-i T1}(d) and P3 = sum K(c, d) e^{-i (T3 - T1)}(d) over a stretch of d
    // on which that order holds (the operator at d annihilates: table 1 or 3).
    auto flush = [&](int c, int code, double2 P1, double2 P3) {
        const int p = tb.perm_of[code];
#pragma unroll
        for (int s1 = 0; s1 < 2; ++s1) {
            const int np = tb.npath[p][s1];
            for (int q = 0; q < np; ++q) {
                const signed char* tq = tb.tab[p][s1][q];
                double2 f = cmul2(fac[tq[0]][a], fac[tq[2]][c]);
                f = cmul2(f, fac[tq[3]][b]);
                f = cmul2(f, tq[1] == 1 ? P1 : P3);
                // G^II carries (-i)^2 = -1, so part = - K G^II adds + w f
                const double w = tb.amp[p][s1][q] * pw[tb.nu[p][s1][q]];
                acc_r += w * f.x;
                acc_i += w * f.y;
            }
        }
    };
    // With (a, b, c) fixed the contour order depends on d only through
    // d > a, d <= c and d <= b (keys: later contour point first, a creation
    // operator later than an annihilation operator at the same point): the
    // cuts after d = a, b and c split [0, N_t) into at most four stretches of
    // constant order, and each stretch's d-sums are differences of the row's
    // prefix sums.  O(N_t^3) per site.
    for (int c = 0; c < n_t; ++c) {
        // Row c times the d factors, one element per thread (N_t <= 256).
        {
            const int d = tid;
            double2 u1 = make_double2(0.0, 0.0), u3 = u1;
            if (d < n_t) {
                const double2 k = Ki[(size_t)c * n_t + d];
                u1 = cmul2(k, fac[1][d]);
                u3 = cmul2(k, fac[3][d]);
            }
            __syncthreads();              // the previous row's sums are no longer read
            pz[0][d + 1] = u1.x;
            pz[1][d + 1] = u1.y;
            pz[2][d + 1] = u3.x;
            pz[3][d + 1] = u3.y;
            if (d < 4) pz[d][0] = 0.0;
        }
        __syncthreads();
        // Inclusive scans: wave w scans array w in chunks of 64 with a carry.
        {
            double carry = 0.0;
            for (int c0 = 0; c0 < n_t; c0 += 64) {
                double v = pz[wave][c0 + lane + 1];
#pragma unroll
                for (int k = 1; k < 64; k <<= 1) {
                    const double t = __shfl_up(v, k);
                    if (lane >= k) v += t;
                }
                v += carry;
                pz[wave][c0 + lane + 1] = v;
                carry = __shfl(v, 63);
            }
        }
        __syncthreads();
        if (live) {
            // the pairs without d: (a, c) c >= a, (a, b) b >= a, (c, b) c < b
            const int code_c = ((c >= a) << 1) | ((b >= a) << 2) | ((c < b) << 5);
            // cut points in increasing order (a stretch ends at each)
            int h0 = a, h1 = b, h2 = c;
            if (h0 > h1) { const int t = h0; h0 = h1; h1 = t; }
            if (h1 > h2) { const int t = h1; h1 = h2; h2 = t; }
            if (h0 > h1) { const int t = h0; h0 = h1; h1 = t; }
            const int hs[4] = {h0, h1, h2, n_t - 1};
            int lo = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int h = hs[k];
                if (h < lo) continue;     // repeated cut
                // stretch [lo, h]: d > a, d <= c and d <= b are constant on it
                const int code = code_c | (lo > a) | ((c >= lo) << 3) | ((b >= lo) << 4);
                const double2 P1 = make_double2(pz[0][h + 1] - pz[0][lo], pz[1][h + 1] - pz[1][lo]);
                const double2 P3 = make_double2(pz[2][h + 1] - pz[2][lo], pz[3][h + 1] - pz[3][lo]);
                flush(c, code, P1, P3);
                lo = h + 1;
            }
        }
    }
    if (live) out[(size_t)site * n_t * n_t + e] = make_double2(acc_r, acc_i);
}

// M = K S per site (one thread per (c, b)), the first factor of the
// cumulant's one-particle term S K S.
__global__ __launch_bounds__(kS2Threads)
void ks_kernel(const double2* __restrict__ S, const double2* __restrict__ K,
               double2* __restrict__ M, Geom g) {
    const int site = blockIdx.y;
    const int n_t = g.n_t;
    const size_t per = (size_t)n_t * n_t;
    const int e = blockIdx.x * kS2Threads + threadIdx.x;
    if (e >= n_t * n_t) return;
    const int c = e / n_t, b = e - (e / n_t) * n_t;
    const double2* Si = S + (size_t)site * per;
    const double2* Ki = K + (size_t)site * per;
    double2 acc = make_double2(0.0, 0.0);
    for (int d = 0; d < n_t; ++d) {
        const double2 v = cmul2(Ki[(size_t)c * n_t + d], Si[(size_t)d * n_t + b]);
        acc.x += v.x;
        acc.y += v.y;
    }
    M[(size_t)site * per + e] = acc;
}

// Sigma~ = part + 2 S(a,b) T - (S M)(a,b), T = sum_{c,d} K(c,d) S(d,c) = trace(M):
// one workgroup per (site, 256 outputs), T reduced inside each workgroup.
__global__ __launch_bounds__(kS2Threads)
void sigma2_onebody_kernel(const double2* __restrict__ S, const double2* __restrict__ M,
                           const double2* __restrict__ part, double2* __restrict__ sig,
                           Geom g) {
    __shared__ double red_r[kS2Threads], red_i[kS2Threads];
    const int site = blockIdx.y;
    const int n_t = g.n_t;
    const size_t per = (size_t)n_t * n_t;
    const double2* Si = S + (size_t)site * per;
    const double2* Mi = M + (size_t)site * per;
    double tr = 0.0, ti = 0.0;
    for (int c = threadIdx.x; c < n_t; c += kS2Threads) {
        tr += Mi[(size_t)c * n_t + c].x;
        ti += Mi[(size_t)c * n_t + c].y;
    }
    red_r[threadIdx.x] = tr;
    red_i[threadIdx.x] = ti;
    __syncthreads();
    for (int s = kS2Threads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            red_r[threadIdx.x] += red_r[threadIdx.x + s];
            red_i[threadIdx.x] += red_i[threadIdx.x + s];
        }
        __syncthreads();
    }
    const double2 T = make_double2(red_r[0], red_i[0]);
    const int e = blockIdx.x * kS2Threads + threadIdx.x;
    if (e >= n_t * n_t) return;
    const int a = e / n_t, b = e - (e / n_t) * n_t;
    double2 sks = make_double2(0.0, 0.0);
    for (int c = 0; c < n_t; ++c) {
        const double2 v = cmul2(Si[(size_t)a * n_t + c], Mi[(size_t)c * n_t + b]);
        sks.x += v.x;
        sks.y += v.y;
    }
    const double2 st = cmul2(Si[e], T);
    const double2 p = part[(size_t)site * per + e];
    sig[(size_t)site * per + e] = make_double2(p.x + 2.0 * st.x - sks.x, p.y + 2.0 * st.y - sks.y);
}

// S' = S (S - Sigma~)^-1 S per site: Gauss-Jordan elimination with partial
// pivoting of [S - Sigma~ | S] (one workgroup per site, the augmented matrix
// in the workspace), then the product with S.
__global__ __launch_bounds__(kDressThreads)
void dress_kernel(const double2* __restrict__ S, const double2* __restrict__ sig,
                  double2* __restrict__ aug, double2* __restrict__ S_out, Geom g,
                  int* __restrict__ singular) {
    __shared__ double rmax[kDressThreads];
    __shared__ int ridx[kDressThreads];
    __shared__ int piv_s;
    const int site = blockIdx.x;
    const int n = g.n_t, w = 2 * n;
    const size_t per = (size_t)n * n;
    const double2* Si = S + (size_t)site * per;
    const double2* Gi = sig + (size_t)site * per;
    double2* A = aug + (size_t)site * n * w;                 // [n][2n]
    for (int e = threadIdx.x; e < n * w; e += kDressThreads) {
        const int r = e / w, c = e - (e / w) * w;
        if (c < n) {
            const double2 s = Si[(size_t)r * n + c], x = Gi[(size_t)r * n + c];
            A[e] = make_double2(s.x - x.x, s.y - x.y);
        } else {
            A[e] = Si[(size_t)r * n + (c - n)];
        }
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // pivot: largest |A(r, k)| for r >= k
        double best = -1.0;
        int bi = k;
        for (int r = k + threadIdx.x; r < n; r += kDressThreads) {
            const double2 v = A[(size_t)r * w + k];
            const double m = fabs(v.x) + fabs(v.y);
            if (m > best) {
                best = m;
                bi = r;
            }
        }
        rmax[threadIdx.x] = best;
        ridx[threadIdx.x] = bi;
        __syncthreads();
        for (int s = kDressThreads / 2; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s && rmax[threadIdx.x + s] > rmax[threadIdx.x]) {
                rmax[threadIdx.x] = rmax[threadIdx.x + s];
                ridx[threadIdx.x] = ridx[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            piv_s = ridx[0];
            if (!(rmax[0] > 0.0)) singular[0] = 1;
        }
        __syncthreads();
        const int p = piv_s;
        if (p != k)
            for (int c = threadIdx.x; c < w; c += kDressThreads) {
                const double2 t = A[(size_t)k * w + c];
                A[(size_t)k * w + c] = A[(size_t)p * w + c];
                A[(size_t)p * w + c] = t;
            }
        __syncthreads();
        // scale the pivot row by 1 / A(k, k)
        const double2 pv = A[(size_t)k * w + k];
        const double den = pv.x * pv.x + pv.y * pv.y;
        const double2 inv = den > 0.0 ? make_double2(pv.x / den, -pv.y / den) : make_double2(0, 0);
        __syncthreads();
        for (int c = threadIdx.x; c < w; c += kDressThreads)
            A[(size_t)k * w + c] = cmul2(A[(size_t)k * w + c], inv);
        __syncthreads();
        // eliminate column k from every other row; columns left of k are
        // already zero in the pivot row
        const int wk = w - k - 1;
        for (int e = threadIdx.x; e < n * wk; e += kDressThreads) {
            const int r = e / wk, c = k + 1 + (e - (e / wk) * wk);
            if (r == k) continue;
            const double2 f = A[(size_t)r * w + k];
            const double2 v = cmul2(f, A[(size_t)k * w + c]);
            const double2 o = A[(size_t)r * w + c];
            A[(size_t)r * w + c] = make_double2(o.x - v.x, o.y - v.y);
        }
        __syncthreads();
        for (int r = threadIdx.x; r < n; r += kDressThreads)
            if (r != k) A[(size_t)r * w + k] = make_double2(0.0, 0.0);
        __syncthreads();
    }
    // S' = S Y, Y = right half of A
    for (int e = threadIdx.x; e < n * n; e += kDressThreads) {
        const int r = e / n, c = e - (e / n) * n;
        double2 acc = make_double2(0.0, 0.0);
        for (int q = 0; q < n; ++q) {
            const double2 v = cmul2(Si[(size_t)r * n + q], A[(size_t)q * w + n + c]);
            acc.x += v.x;
            acc.y += v.y;
        }
        S_out[(size_t)site * per + e] = acc;
    }
}

// Linear mixing of eq. Sigmamix, sig <- lam new + (1 - lam) sig, with the
// per-workgroup partial sum of |new - sig|^2 and maximum of |new - sig|.
__global__ __launch_bounds__(256)
void mix_kernel(const double2* __restrict__ fresh, double2* __restrict__ sig, double lam,
                size_t n, double* __restrict__ part) {
    __shared__ double rs[256], rm[256];
    double s2 = 0.0, mx = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const double2 a = fresh[e], b = sig[e];
        const double dr = a.x - b.x, di = a.y - b.y;
        const double m2 = dr * dr + di * di;
        s2 += m2;
        mx = fmax(mx, sqrt(m2));
        if (!(m2 == m2)) mx = m2;                     // keep a NaN
        sig[e] = make_double2(lam * a.x + (1.0 - lam) * b.x, lam * a.y + (1.0 - lam) * b.y);
    }
    rs[threadIdx.x] = s2;
    rm[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            rs[threadIdx.x] += rs[threadIdx.x + s];
            const double o = rm[threadIdx.x + s];
            if (o > rm[threadIdx.x] || !(o == o)) rm[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = rs[0];
        part[2 * blockIdx.x + 1] = rm[0];
    }
}

}  // namespace

hipError_t launch_mix(const double2* fresh, double2* sig, double lam, size_t n, double* part,
                      int n_part, hipStream_t st) {
    hipLaunchKernelGGL(mix_kernel, dim3(n_part), dim3(256), 0, st, fresh, sig, lam, n, part);
    return hipGetLastError();
}

hipError_t launch_sigma2(const Geom& g, const double* V, const double* U, const double* J,
                         const double2* S, const double2* G_loc_all, double2* K, double2* part,
                         double2* M, double2* sig, hipStream_t st) {
    hipLaunchKernelGGL(k_build_kernel, dim3(2048), dim3(256), 0, st, G_loc_all, J, K, g);
    const dim3 grid((g.n_t * g.n_t + kS2Threads - 1) / kS2Threads, g.n_r);
    static const PathTable paths = build_path_table();
    hipLaunchKernelGGL(sigma2_pair_kernel, grid, dim3(kS2Threads), 0, st, K, V, U, part, g, paths);
    hipLaunchKernelGGL(ks_kernel, grid, dim3(kS2Threads), 0, st, S, K, M, g);
    hipLaunchKernelGGL(sigma2_onebody_kernel, grid, dim3(kS2Threads), 0, st, S, M, part, sig, g);
    return hipGetLastError();
}

hipError_t launch_dress(const Geom& g, const double2* S, const double2* sig, double2* aug,
                        double2* S_out, int* singular, hipStream_t st) {
    hipLaunchKernelGGL(dress_kernel, dim3(g.n_r), dim3(kDressThreads), 0, st, S, sig, aug, S_out, g,
                       singular);
    return hipGetLastError();
}

}  // namespace scd

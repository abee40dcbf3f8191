// Point-group reduction of the source columns (App. A of arXiv:1309.5994):
// on a trap invariant under the lattice's point group (C4v for a square
// lattice about its centre, C2v for a rectangle), G(g(i), g(j)) = G(i, j) for
// every group element g, so only one source per orbit (its representative)
// needs solving; the columns of every other source s = g(r) are those of r
// with the target sites permuted by g^-1 and the neighbour slots relabelled.
//
// Host side: the group's site permutations, the orbits and the slot maps.
// Device side: the invariance check of S and the extraction that writes the
// kept blocks of every requested source straight from the representatives'
// block iterate.
#include <utility>

#include "internal.h"

namespace scd {
namespace {

// max over sites and entries of |S_i - S_perm(i)| (real and imaginary parts),
// per-workgroup partial maxima.
__global__ __launch_bounds__(256)
void sym_check_kernel(const double2* __restrict__ S, const int* __restrict__ perm, int n_r,
                      int n_t, double* __restrict__ part) {
    __shared__ double red[256];
    const size_t per = (size_t)n_t * n_t;
    const size_t total = (size_t)n_r * per;
    double m = 0.0;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / per);
        const size_t off = e - (size_t)i * per;
        const double2 a = S[e];
        const double2 b = S[(size_t)perm[i] * per + off];
        const double d = fmax(fabs(a.x - b.x), fabs(a.y - b.y));
        m = (d > m || d != d) ? d : m;     // keep a NaN
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            const double o = red[threadIdx.x + s];
            if (o > red[threadIdx.x] || o != o) red[threadIdx.x] = o;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Kept blocks of the requested sources whose representatives sit in the
// current block.  For entry q of the list: requested index s = req[q], column
// block position lr of its representative r = src_blk[lr], group element g
// with s = g(r):
//   G_loc[s]        = X[r][:, lr N_t + :]
//   G_nn[s][d]      = X[nbr_slot(s,d)(r)][:, lr N_t + :]   (zero for no neighbour)
//   G_cols[i][:, s] = X[g^-1(i)][:, lr N_t + :]
__global__ __launch_bounds__(256)
void extract_sym_kernel(const double2* __restrict__ X, int ldx, const int* __restrict__ src_blk,
                        const int* __restrict__ req, const int* __restrict__ req_lr,
                        const int* __restrict__ req_g, const int* __restrict__ req_slot,
                        const int* __restrict__ perm_inv, int n_req, int n_src,
                        double2* __restrict__ G_cols, double2* __restrict__ G_loc,
                        double2* __restrict__ G_nn, Geom g) {
    const int n_t = g.n_t;
    const size_t nn = (size_t)n_t * n_t;
    const size_t per_src = 5 * nn + (G_cols ? (size_t)g.n_r * nn : 0);
    const size_t total = (size_t)n_req * per_src;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int q = (int)(e / per_src);
        const size_t f = e - (size_t)q * per_src;
        const int s = req[q], lr = req_lr[q];
        const int r = src_blk[lr];
        const int b = (int)(f % n_t);
        const int a = (int)((f / n_t) % n_t);
        const size_t col = (size_t)lr * n_t + b;
        if (f < 5 * nn) {
            const int slot = (int)(f / nn);
            int k = r;
            if (slot > 0) {
                const int d = req_slot[4 * q + slot - 1];
                int nb[4];
                site_neighbours(r, g.Lx, g.Ly, g.periodic, nb);
                k = d >= 0 ? nb[d] : -1;
            }
            const double2 v = k >= 0 ? X[((size_t)k * g.mp + a) * ldx + col] : make_double2(0.0, 0.0);
            if (slot == 0)
                G_loc[((size_t)s * n_t + a) * n_t + b] = v;
            else if (G_nn)
                G_nn[(((size_t)s * 4 + slot - 1) * n_t + a) * n_t + b] = v;
        } else {
            const int i = (int)((f - 5 * nn) / nn);
            const int k = perm_inv[(size_t)req_g[q] * g.n_r + i];
            G_cols[((size_t)i * n_t + a) * ((size_t)n_src * n_t) + (size_t)s * n_t + b] =
                X[((size_t)k * g.mp + a) * ldx + col];
        }
    }
}

}  // namespace

SymGroup lattice_group(const Geom& g) {
    SymGroup G;
    const int Lx = g.Lx, Ly = g.Ly;
    const int n_el = Lx == Ly ? 8 : 4;
    G.n_el = n_el;
    G.perm.assign((size_t)n_el * g.n_r, 0);
    G.perm_inv.assign((size_t)n_el * g.n_r, 0);
    for (int e = 0; e < n_el; ++e) {
        for (int x = 0; x < Lx; ++x) {
            for (int y = 0; y < Ly; ++y) {
                int u = x, v = y;
                if (e & 1) u = Lx - 1 - u;          // mirror x
                if (e & 2) v = Ly - 1 - v;          // mirror y
                if (e & 4) std::swap(u, v);         // diagonal (square lattices)
                const int i = x * Ly + y, j = u * Ly + v;
                G.perm[(size_t)e * g.n_r + i] = j;
                G.perm_inv[(size_t)e * g.n_r + j] = i;
            }
        }
    }
    // Orbit representative (smallest site index) and an element taking it to i.
    G.rep.assign(g.n_r, -1);
    G.elem.assign(g.n_r, 0);
    for (int i = 0; i < g.n_r; ++i) {
        if (G.rep[i] >= 0) continue;
        for (int e = 0; e < n_el; ++e) {
            const int j = G.perm[(size_t)e * g.n_r + i];
            if (G.rep[j] < 0) {
                G.rep[j] = i;
                G.elem[j] = e;
            }
        }
    }
    return G;
}

int sym_slot(const SymGroup& G, const Geom& g, int s, int d) {
    int nb_s[4], nb_r[4];
    site_neighbours(s, g.Lx, g.Ly, g.periodic, nb_s);
    if (nb_s[d] < 0) return -1;
    const int r = G.rep[s];
    const int k = G.perm_inv[(size_t)G.elem[s] * g.n_r + nb_s[d]];
    site_neighbours(r, g.Lx, g.Ly, g.periodic, nb_r);
    for (int q = 0; q < 4; ++q)
        if (nb_r[q] == k) return q;
    return -2;   // not a symmetry of the neighbour structure
}

hipError_t launch_sym_check(const double2* S, const int* perm, const Geom& g, double* part,
                            int n_part, hipStream_t st) {
    hipLaunchKernelGGL(sym_check_kernel, dim3(n_part), dim3(256), 0, st, S, perm, g.n_r, g.n_t,
                       part);
    return hipGetLastError();
}

hipError_t launch_extract_sym(const Geom& g, const double2* X, int ldx, const int* src_blk,
                              const int* req, const int* req_lr, const int* req_g,
                              const int* req_slot, const int* perm_inv, int n_req, int n_src,
                              double2* G_cols, double2* G_loc, double2* G_nn, hipStream_t st) {
    if (n_req == 0) return hipSuccess;
    hipLaunchKernelGGL(extract_sym_kernel, dim3(4096), dim3(256), 0, st, X, ldx, src_blk, req,
                       req_lr, req_g, req_slot, perm_inv, n_req, n_src, G_cols, G_loc, G_nn, g);
    return hipGetLastError();
}

}  // namespace scd

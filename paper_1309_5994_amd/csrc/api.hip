// C-ABI entry points of libscdyson: argument validation, workspace layout,
// column-block scheduling and the host side of the convergence loop.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace scd;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* where) {
    return fail(SCD_EHIP, "%s: %s", where, hipGetErrorString(e));
}

#define SCD_HIP(call, where)                         \
    do {                                             \
        hipError_t e_ = (call);                      \
        if (e_ != hipSuccess) return hip_fail(e_, where); \
    } while (0)

int check_problem(const scd_problem* p, int max_nt, Geom* g) {
    if (!p) return fail(SCD_EINVAL, "problem is NULL");
    if (p->Lx < 1 || p->Ly < 1) return fail(SCD_EINVAL, "lattice extent must be >= 1");
    if ((int64_t)p->Lx * p->Ly > 65535) return fail(SCD_EINVAL, "at most 65535 sites");
    if (p->periodic != 0 && p->periodic != 1) return fail(SCD_EINVAL, "periodic must be 0 or 1");
    if (p->periodic && (p->Lx < 3 || p->Ly < 3))
        return fail(SCD_EINVAL, "periodic lattices need Lx, Ly >= 3");
    if (p->n_real < 1 || p->n_imag < 1) return fail(SCD_EINVAL, "n_real and n_imag must be >= 1");
    const int64_t n_t = 2 * (int64_t)p->n_real + p->n_imag;
    if (n_t > max_nt) return fail(SCD_EINVAL, "contour has %lld points, at most %d supported",
                                  (long long)n_t, max_nt);
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(SCD_EINVAL, "dt must be > 0");
    if (!(p->beta > 0.0) || !std::isfinite(p->beta)) return fail(SCD_EINVAL, "beta must be > 0");
    if (!std::isfinite(p->mu) || !std::isfinite(p->t_min))
        return fail(SCD_EINVAL, "mu and t_min must be finite");
    g->Lx = p->Lx;
    g->Ly = p->Ly;
    g->periodic = p->periodic;
    g->n_r = p->Lx * p->Ly;
    g->n_real = p->n_real;
    g->n_imag = p->n_imag;
    g->n_t = (int)n_t;
    g->mt = (g->n_t + kTile - 1) / kTile;
    g->mp = g->mt * kTile;
    g->dt = p->dt;
    g->beta = p->beta;
    g->mu = p->mu;
    g->t_min = p->t_min;
    g->dtau = p->beta / p->n_imag;
    return SCD_OK;
}

struct Layout {
    int ldx, ntn, nwg;
    size_t off_st, off_st32, off_x0, off_x1, off_r32, off_d0, off_d1, off_partial, off_slot,
        off_src, off_order, total;
};

bool lattice_bipartite(const Geom& g) { return !g.periodic || (g.Lx % 2 == 0 && g.Ly % 2 == 0); }

// Workspace: St (FP64 operand) and one FP64 iterate, updated in place by
// red-black sweeps; refined paths: + the low-precision operand (complex64
// St32 for FP32, six bf16 planes for BF16x3), the complex64 residual and one
// correction.  A lattice that is not bipartite (periodic with an odd extent)
// sweeps Jacobi-style and needs a second FP64 iterate (second correction).
Layout layout(const Geom& g, int n_src, int block_sites, int prec) {
    Layout L;
    const int bs = block_sites < n_src ? block_sites : n_src;
    const bool rb = lattice_bipartite(g);
    L.ldx = ((bs * g.n_t + kColsPerWG - 1) / kColsPerWG) * kColsPerWG;
    L.ntn = L.ldx / kColsPerWG;
    L.nwg = g.n_r * L.ntn;
    const size_t it64 = (size_t)g.n_r * g.mp * L.ldx * sizeof(double2);
    const size_t it32 = (size_t)g.n_r * g.mp * L.ldx * sizeof(float2);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.off_st = take((size_t)g.n_r * g.mp * g.mp * sizeof(double2));
    L.off_x0 = take(it64);
    L.off_x1 = L.off_st32 = L.off_r32 = L.off_d0 = L.off_d1 = 0;
    if (prec == SCD_PREC_FP64) {
        if (!rb) L.off_x1 = take(it64);
    } else {
        L.off_st32 = take(prec == SCD_PREC_BF16X3 ? bf3_operand_bytes(g)
                                                  : (size_t)g.n_r * g.mp * g.mp * sizeof(float2));
        L.off_r32 = take(it32);
        L.off_d0 = take(it32);
        if (!rb) L.off_d1 = take(it32);
    }
    L.off_partial = take((size_t)L.nwg * 3 * sizeof(double));
    L.off_slot = take(4 * sizeof(unsigned long long));
    L.off_src = take((size_t)n_src * sizeof(int32_t));
    L.off_order = take((size_t)g.n_r * sizeof(int32_t));
    L.total = off;
    return L;
}

double bits_to_double(unsigned long long u) {
    double d;
    std::memcpy(&d, &u, sizeof d);
    return d;
}

struct BlockResult {
    double2* X = nullptr;   // buffer holding the final iterate
    int sweeps = 0;
    double err = 0.0, rho = 0.0;
};

// Launch timing without a host sync per launch: events are recorded around
// each launch and read back at the next convergence check.
struct LaunchTimer {
    std::vector<hipEvent_t> ev;
    size_t used = 0;
    ~LaunchTimer() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
    hipError_t mark(hipStream_t st) {
        if (used == ev.size()) {
            hipEvent_t e;
            hipError_t rc = hipEventCreate(&e);
            if (rc != hipSuccess) return rc;
            ev.push_back(e);
        }
        return hipEventRecord(ev[used++], st);
    }
    // Sum of (end - begin) over the recorded pairs; the stream must be synchronised.
    hipError_t drain(double* seconds) {
        double sum = 0.0;
        for (size_t k = 0; k + 1 < used; k += 2) {
            float ms = 0.0f;
            hipError_t rc = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            if (rc != hipSuccess) return rc;
            sum += 1e-3 * ms;
        }
        used = 0;
        *seconds = sum;
        return hipSuccess;
    }
};

// When to measure convergence: every sweep at first, then at points predicted
// from the measured contraction rate (see schedule), then every sweep.
struct CheckPlan {
    int last_n = 0, next = 1;
    double last_e = 0.0, rho = 0.0;
    bool due(int n) const { return n <= 3 || n >= next; }
    // A measured increment e at sweep n: updates the rate estimate.
    void record(int n, double e) {
        if (last_n > 0 && last_e > 0.0 && e > 0.0)
            rho = std::pow(e / last_e, 1.0 / (double)(n - last_n));
        last_n = n;
        last_e = e;
    }
    // Next check: after 60 % of the sweeps predicted to bring e below target
    // (the longer baseline sharpens the rate), every sweep once 2 or fewer remain.
    void schedule(int n, double e, double target) {
        int k = 1;
        if (rho > 0.0 && rho < 1.0 && e > target && target > 0.0)
            k = (int)std::ceil(std::log(target / e) / std::log(rho));
        k = std::max(1, std::min(k, 64));
        next = n + (k <= 2 ? 1 : std::max(1, (int)(0.6 * k)));
    }
};

// Device buffers of the batched GMRES of one column block (see gm_layout).
struct GmBufs {
    double2* u;          // iterate
    double2* Q;          // basis v_0 .. v_restart, qstride elements apart
    size_t qstride;
    double2 *pa, *pb;    // Gram-Schmidt dot partials [nch][kMaxBasis][ldx]
    double* pn;          // norm partials [nch][ldx]
    double* sig;         // [kMaxBasis + 1][ldx]
    double2* R;          // [kMaxBasis][kMaxBasis][ldx]
    double* cs;          // [kMaxBasis][ldx]
    double2* sn;         // [kMaxBasis][ldx]
    double2* gv;         // [kMaxBasis + 1][ldx]
    double2* y;          // [kMaxBasis][ldx]
    double* x0n;         // [ldx]
    int rows, ldx, nch, chunk_rows;
};

// Host side of the sweep loops of one column block.
struct Solver {
    Geom g;
    hipStream_t st;
    scd_stats* stats;
    double2* St;
    void* St32;         // low-precision operand (complex64, or BF16x3 planes)
    bool bf3 = false;   // correction sweeps on the BF16x3 engine
    const double2* S;
    double* partial;
    unsigned long long* slot;
    int nwg;
    const int* colour_sites[2] = {nullptr, nullptr};   // device site lists (red-black)
    int n_colour[2] = {0, 0};
    const int* all_sites = nullptr;   // device list of all n_r sites (launches over every site)
    LaunchTimer t64, t32, ts;         // FP64 sweeps, low-precision sweeps, streaming passes
    std::vector<double> within[3];   // (target, source) pairs within distance d, cumulative:
                                     // [0] all targets, [1] even-colour, [2] odd-colour targets

    void pair_counts(const int32_t* src_host, int bs) {
        for (auto& w : within) w.assign(g.Lx + g.Ly + 1, 0.0);
        for (int s = 0; s < bs; ++s) {
            const int j = src_host[s];
            const int xj = j / g.Ly, yj = j % g.Ly;
            for (int i = 0; i < g.n_r; ++i) {
                const int xi = i / g.Ly, yi = i % g.Ly;
                int dx = std::abs(xi - xj), dy = std::abs(yi - yj);
                if (g.periodic) {
                    dx = std::min(dx, g.Lx - dx);
                    dy = std::min(dy, g.Ly - dy);
                }
                within[0][dx + dy] += 1.0;
                within[1 + (xi + yi) % 2][dx + dy] += 1.0;
            }
        }
        for (auto& w : within)
            for (size_t d = 1; d < w.size(); ++d) w[d] += w[d - 1];
    }
    // Algorithmic flops of a launch whose output reaches lattice distance
    // `radius` on the targets of `which` (0 all, 1 even, 2 odd colour).
    int trunc = -1;    // truncation radius of the solve, or -1
    double sweep_flops(int radius, int cols_per_src, int which = 0) const {
        if (trunc >= 0 && radius > trunc) radius = trunc;
        const std::vector<double>& w = within[which];
        const size_t last = w.size() - 1;
        const double pairs = w[(size_t)radius < last ? (size_t)radius : last];
        return 8.0 * g.n_t * (double)g.n_t * (double)cols_per_src * pairs;
    }
    // Fold the per-workgroup partials of the last sweep and collect the launch
    // timings; returns SCD_OK or SCD_EHIP.
    int reduce(double out[3], int n_parts = 0) {
        SCD_HIP(hipMemsetAsync(slot, 0, 4 * sizeof(unsigned long long), st), "slot clear");
        SCD_HIP(launch_reduce_max3(partial, n_parts > 0 ? n_parts : nwg, slot, st),
                "reduce launch");
        unsigned long long h[3];
        SCD_HIP(hipMemcpyAsync(h, slot, sizeof h, hipMemcpyDeviceToHost, st), "slot copy");
        SCD_HIP(hipStreamSynchronize(st), "sweep sync");
        for (int q = 0; q < 3; ++q) out[q] = bits_to_double(h[q]);
        double s64 = 0.0, s32 = 0.0, sst = 0.0;
        SCD_HIP(t64.drain(&s64), "event time");
        SCD_HIP(t32.drain(&s32), "event time");
        SCD_HIP(ts.drain(&sst), "event time");
        stats->sweep_kernel_seconds += s64;
        stats->lowp_kernel_seconds += s32;
        stats->stream_kernel_seconds += sst;
        return SCD_OK;
    }
    bool red_black() const { return colour_sites[0] != nullptr; }

    // One sweep X <- X0 + St^T N(X) (FP64) or D <- R + St32^T N(D) (FP32
    // correction): red-black in place, or Jacobi into `nxt`.  `half` counts the
    // launches already applied (the light-cone radius).
    int sweep(SweepArgs a, bool fp32, const int* src_blk, void* cur, void* nxt, const void* R32,
              int cps, int* half) {
        const bool cone = a.lc_sweep >= 0;
        const int launches = red_black() ? 2 : 1;
        int off = 0;
        for (int c = 0; c < launches; ++c) {
            a.sites = red_black() ? colour_sites[c] : all_sites;
            a.n_sites = red_black() ? n_colour[c] : g.n_r;
            a.part_off = off;
            a.lc_sweep = cone ? *half : -1;
            void* out = red_black() ? cur : nxt;
            LaunchTimer& tm = fp32 ? t32 : t64;
            SCD_HIP(tm.mark(st), "event record");
            if (fp32)
                SCD_HIP(bf3 ? launch_correct_bf3(g, a, St32, src_blk, R32, cur, out, partial, st)
                            : launch_correct_f32(g, a, St32, src_blk, R32, cur, out, partial, st),
                        "correct launch");
            else
                SCD_HIP(launch_sweep_f64(g, a, St, S, src_blk, (const double2*)cur,
                                         (double2*)out, partial, st),
                        "sweep launch");
            SCD_HIP(tm.mark(st), "event record");
            if (fp32)
                stats->lowp_launches++;
            else
                stats->sweep_launches++;
            stats->gemm_flops += sweep_flops(cone ? *half + 1 : 1 << 20, cps,
                                             red_black() ? 1 + c : 0);
            off += a.n_sites * a.ntn;
            ++*half;
        }
        return SCD_OK;
    }

    // FP64 sweeps until the relative increment e_n and its contraction-corrected
    // error estimate e_n rho / (1 - rho) are below tol.
    int solve_fp64(SweepArgs a, const int* src_blk, double2* X, double2* Xn, double tol,
                   int max_iter, BlockResult* res) {
        const int cps = a.x0_kind == X0_BLOCK ? g.n_t : 1;
        double e_n = 0.0, d_prev = 0.0;
        int grow = 0, n = 0, code = SCD_ENOTCONV, half = 0;
        CheckPlan plan;
        void* cur = X;
        void* nxt = Xn;
        for (n = 1; n <= max_iter; ++n) {
            a.check = (plan.due(n) || n == max_iter) ? 1 : 0;
            if (sweep(a, false, src_blk, cur, nxt, nullptr, cps, &half)) return SCD_EHIP;
            if (!red_black()) std::swap(cur, nxt);
            stats->fp64_sweeps++;
            if (!a.check) continue;
            double r[3];
            if (reduce(r)) return SCD_EHIP;
            if (r[2] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1])) {
                code = fail(SCD_ENAN, "NaN or Inf in the iterate at sweep %d", n);
                break;
            }
            e_n = r[1] > 0.0 ? r[0] / r[1] : 0.0;
            if (e_n == 0.0) {
                code = SCD_OK;
                break;
            }
            plan.record(n, e_n);
            const double rho = plan.rho;
            if (e_n <= tol && n >= 2 &&
                (e_n <= 1e-2 * tol || (rho < 1.0 && e_n * rho / (1.0 - rho) <= tol))) {
                code = SCD_OK;
                break;
            }
            plan.schedule(n, e_n,
                          (rho > 0.0 && rho < 1.0) ? tol * std::min(1.0, (1.0 - rho) / rho) : tol);
            // A convergent Dyson series has shrinking increments; a divergent one
            // grows them geometrically (the relative increment stays O(1)).
            grow = (n >= 2 && r[0] > d_prev) ? grow + 1 : 0;
            if (grow > 0) plan.next = n + 1;
            if (grow >= 8) {
                code = fail(SCD_EDIVERGED,
                            "sweep increments grew 8 times in a row (|dX|=%g, sweep %d)", r[0], n);
                break;
            }
            d_prev = r[0];
        }
        if (code == SCD_ENOTCONV) {
            double r[3];
            if (reduce(r)) return SCD_EHIP;
        }
        res->X = (double2*)cur;
        res->sweeps = n > max_iter ? max_iter : n;
        res->err = e_n;
        res->rho = plan.rho;
        return code;
    }

    // Iterative refinement: FP64 residual R = X0 + St^T N(X) - X (complex64
    // output), FP32-MFMA correction sweeps D <- R + St^T N(D) (red-black in
    // place, or Jacobi between D0 and D1) to the relative increment the outer
    // target needs (at most 0.1, at least the FP32 floor 1e-6, or until
    // stagnation), then X += D in FP64.  Stops when the relative FP64
    // residual, divided by (1 - rho), is below tol.
    int solve_mixed(SweepArgs a, const int* src_blk, double2* X, void* R32, void* D0, void* D1,
                    double tol, int max_iter, BlockResult* res) {
        const int cps = a.x0_kind == X0_BLOCK ? g.n_t : 1;
        const size_t n_elem = (size_t)g.n_r * g.mp * a.ldx;
        const size_t bytes32 = n_elem * sizeof(float2);
        // R and D0 start at zero: tiles beyond the light cone are never written.
        SCD_HIP(hipMemsetAsync(R32, 0, bytes32, st), "clear");
        SCD_HIP(hipMemsetAsync(D0, 0, bytes32, st), "clear");
        if (D1) SCD_HIP(hipMemsetAsync(D1, 0, bytes32, st), "clear");
        const bool cone = a.lc_sweep >= 0;
        int radius_x = 0;           // lattice distance the iterate reaches
        double rho = 0.0, e_r = 0.0, d_prev = 0.0;
        int outer = 0, code = SCD_ENOTCONV, grow = 0;
        const int max_inner = 1000;
        for (outer = 1; outer <= max_iter; ++outer) {
            a.sites = all_sites;
            a.n_sites = g.n_r;
            a.part_off = 0;
            a.check = 1;
            a.lc_sweep = cone ? radius_x : -1;
            SCD_HIP(t64.mark(st), "event record");
            // The residual kernel also writes R into D0, the correction's start
            // (D_0 = R): outside its light cone both stay zero, as D0 was never
            // written there by earlier correction sweeps (their cone is smaller).
            a.out2 = D0;
            SCD_HIP(launch_residual_f64(g, a, St, S, src_blk, X, R32, partial, st),
                    "residual launch");
            a.out2 = nullptr;
            SCD_HIP(t64.mark(st), "event record");
            double r[3];
            if (reduce(r)) return SCD_EHIP;
            stats->fp64_sweeps++;
            stats->sweep_launches++;
            stats->gemm_flops += sweep_flops(cone ? radius_x + 1 : 1 << 20, cps);
            if (r[2] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1])) {
                code = fail(SCD_ENAN, "NaN or Inf in the FP64 residual at refinement step %d",
                            outer);
                break;
            }
            e_r = r[1] > 0.0 ? r[0] / r[1] : 0.0;
            if (e_r == 0.0 || (outer >= 2 && rho < 1.0 && e_r / (1.0 - rho) <= tol)) {
                code = SCD_OK;
                break;
            }
            grow = (outer >= 2 && r[0] > d_prev) ? grow + 1 : 0;
            if (grow >= 3) {
                code = fail(SCD_EDIVERGED, "FP64 residual grew 3 refinement steps in a row (%g)",
                            r[0]);
                break;
            }
            d_prev = r[0];
            if (outer == max_iter) break;
            // Correction sweeps from D_0 = R, solved only as accurately as the
            // outer target needs: the corrected X is off by about
            // eta |R| / (1 - rho) for a relative correction accuracy eta.
            const double rho_g = (rho > 0.0 && rho < 1.0) ? rho : 0.5;
            const double floor = bf3 ? 3e-5 : 1e-6;   // accuracy of the correction engine
            const double inner_tol =
                std::min(0.1, std::max(floor, 0.3 * tol * (1.0 - rho_g) / e_r));
            const int radius_r = radius_x + 1;
            void* dc = D0;
            void* dn = D1;
            double e_prev = 0.0;
            int j = 0, stall = 0, half = radius_r;
            CheckPlan plan;
            for (j = 1; j <= max_inner; ++j) {
                a.check = (plan.due(j) || j == max_inner) ? 1 : 0;
                if (sweep(a, true, src_blk, dc, dn, R32, cps, &half)) return SCD_EHIP;
                if (!red_black()) std::swap(dc, dn);
                stats->lowp_sweeps++;
                if (!a.check) continue;
                if (reduce(r)) return SCD_EHIP;
                if (r[2] != 0.0 || !std::isfinite(r[0]) || !std::isfinite(r[1])) {
                    code = fail(SCD_ENAN, "NaN or Inf in an FP32 correction sweep");
                    break;
                }
                const double e_in = r[1] > 0.0 ? r[0] / r[1] : 0.0;
                plan.record(j, e_in);
                plan.schedule(j, e_in, inner_tol);
                if (plan.rho > 0.0 && plan.rho < 1.0) rho = plan.rho;
                stall = (j >= 2 && e_in >= e_prev) ? stall + 1 : 0;
                if (stall > 0) plan.next = j + 1;
                e_prev = e_in;
                if (e_in <= inner_tol || stall >= 3) break;
            }
            if (code == SCD_ENAN) break;
            SCD_HIP(launch_axpy_f32_to_f64(X, dc, n_elem, st), "axpy launch");
            radius_x = half;
        }
        res->X = X;
        res->sweeps = outer > max_iter ? max_iter : outer;
        res->err = e_r;
        res->rho = rho;
        return code;
    }

    // Elements (row x column) of the streaming passes' workgroups whose
    // nearest (site, source) pair lies within lattice distance d, cumulative
    // in d: the part of a Krylov vector a pass with light-cone radius d moves.
    std::vector<double> gs_area;
    void gs_area_table(const GsPass& p, const int32_t* src_host) {
        gs_area.assign(g.Lx + g.Ly + 2, 0.0);
        const int spc = p.chunk_rows / g.mp;
        for (int c_lo = 0; c_lo < p.ldx; c_lo += 64) {
            const int c_hi = std::min(p.ldx, c_lo + 64) - 1;
            const int s_lo = c_lo / g.n_t, s_hi = std::min(c_hi / g.n_t, p.bs - 1);
            if (s_lo >= p.bs) continue;
            for (int i_lo = 0; i_lo < g.n_r; i_lo += spc) {
                const int i_hi = std::min(g.n_r, i_lo + spc) - 1;
                int dmin = 1 << 30;
                for (int s = s_lo; s <= s_hi; ++s) {
                    const int j = src_host[s];
                    for (int i = i_lo; i <= i_hi; ++i) {
                        int dx = std::abs(i / g.Ly - j / g.Ly), dy = std::abs(i % g.Ly - j % g.Ly);
                        if (g.periodic) {
                            dx = std::min(dx, g.Lx - dx);
                            dy = std::min(dy, g.Ly - dy);
                        }
                        dmin = std::min(dmin, dx + dy);
                    }
                }
                gs_area[std::min<int>(dmin, (int)gs_area.size() - 1)] +=
                    (double)(i_hi - i_lo + 1) * g.mp * (c_hi - c_lo + 1);
            }
        }
        for (size_t d = 1; d < gs_area.size(); ++d) gs_area[d] += gs_area[d - 1];
    }

    // One streaming pass, timed and counted; `vectors` = Krylov-sized vectors
    // it reads plus writes, over the workgroups inside its light cone.
    int gs(int mode, GsPass p, int vectors) {
        SCD_HIP(ts.mark(st), "event record");
        SCD_HIP(launch_gs(mode, p, st), "Gram-Schmidt launch");
        SCD_HIP(ts.mark(st), "event record");
        stats->stream_launches++;
        const double area = p.radius < 0 ? (double)p.rows * p.ldx
                                         : gs_area[std::min<size_t>(p.radius, gs_area.size() - 1)];
        stats->stream_bytes += (double)vectors * area * sizeof(double2);
        return SCD_OK;
    }

    // Batched GMRES(restart) of one column block (App. C), all columns in lock
    // step from u = X0: at each (re)start the FP64 residual z = X0 + St^T N(u) - u
    // (the preconditioned residual S e - (I - S D) u) becomes v_0; each Arnoldi
    // step is one batched matvec w = St^T N(v_d) (sweep kernel without X0)
    // followed by classical Gram-Schmidt applied twice and the Givens update of
    // every column's Hessenberg system.  A cycle ends after `restart` steps or
    // once the largest rotated residual |g_{d+1}| / |X0| over the columns is at
    // most tol; the block has converged when the recomputed FP64 residual
    // |z| / |X0| of every column is at most tol.
    int solve_gmres(SweepArgs a, const int* src_blk, const int32_t* src_host, const GmBufs& b,
                    int restart, double tol, int max_iter, BlockResult* res) {
        const int cps = g.n_t;
        const bool cone = a.lc_sweep >= 0;
        const size_t vbytes = (size_t)b.rows * b.ldx * sizeof(double2);
        const int ngw = (b.ldx + 255) / 256;
        GsPass p{};
        p.Q = b.Q;
        p.qstride = b.qstride;
        p.sig = b.sig;
        p.rows = b.rows;
        p.ldx = b.ldx;
        p.chunk_rows = b.chunk_rows;
        p.pnorm = b.pn;
        p.src_blk = src_blk;
        p.radius = -1;
        p.bs = a.bs;
        p.n_t = g.n_t;
        p.mp = g.mp;
        p.Lx = g.Lx;
        p.Ly = g.Ly;
        p.periodic = g.periodic;
        gs_area_table(p, src_host);
        const size_t pstride = (size_t)kMaxBasis * b.ldx;
        GivensArgs ga{};
        ga.pa = b.pa;
        ga.pb = b.pb;
        ga.pn = b.pn;
        ga.nch = b.nch;
        ga.ldx = b.ldx;
        ga.sig = b.sig;
        ga.R = b.R;
        ga.cs = b.cs;
        ga.sn = b.sn;
        ga.gv = b.gv;
        ga.x0n = b.x0n;
        ga.part = partial;

        // |X0| per column (u = X0 on entry).
        {
            GsPass q = p;
            q.k = 0;
            q.w = b.u;
            q.radius = cone ? 0 : -1;
            if (gs(GS_NORM, q, 1)) return SCD_EHIP;
            SCD_HIP(launch_colnorm(b.pn, b.nch, b.ldx, b.x0n, st), "column norm launch");
        }
        int radius_u = 0, n = 0, cleared = 0, code = SCD_ENOTCONV;
        double e = 0.0, e0 = 0.0;
        double r[3];
        auto clear_basis = [&](int j) -> int {
            // Tiles beyond the light cone are never written by the matvec.
            if (j < cleared) return SCD_OK;
            SCD_HIP(hipMemsetAsync(b.Q + (size_t)j * b.qstride, 0, vbytes, st), "basis clear");
            cleared = j + 1;
            return SCD_OK;
        };
        for (;;) {
            // (Re)start: v_0 = z = X0 + St^T N(u) - u, sig_0 = 1 / |z| per column.
            if (clear_basis(0)) return SCD_EHIP;
            a.sites = all_sites;
            a.n_sites = g.n_r;
            a.part_off = 0;
            a.check = 1;
            a.no_x0 = 0;
            a.out_f64 = 1;
            a.lc_sweep = cone ? radius_u : -1;
            SCD_HIP(t64.mark(st), "event record");
            SCD_HIP(launch_residual_f64(g, a, St, S, src_blk, b.u, b.Q, partial, st),
                    "residual launch");
            SCD_HIP(t64.mark(st), "event record");
            a.out_f64 = 0;
            stats->fp64_sweeps++;
            stats->sweep_launches++;
            stats->gemm_flops += sweep_flops(cone ? radius_u + 1 : 1 << 20, cps);
            {
                GsPass q = p;
                q.k = 0;
                q.w = b.Q;
                q.radius = cone ? radius_u + 1 : -1;
                if (gs(GS_NORM, q, 1)) return SCD_EHIP;
            }
            ga.d = -1;
            SCD_HIP(launch_givens(ga, st), "Givens launch");
            if (reduce(r, ngw)) return SCD_EHIP;
            if (r[2] != 0.0 || !std::isfinite(r[0])) {
                code = fail(SCD_ENAN, "NaN or Inf in the GMRES residual after %d steps", n);
                break;
            }
            e = r[0];
            if (n == 0) e0 = e;
            if (e <= tol) {
                code = SCD_OK;
                break;
            }
            if (n >= max_iter) break;
            for (int d = 0; d < restart; ++d) {
                double2* v = b.Q + (size_t)d * b.qstride;
                double2* w = b.Q + (size_t)(d + 1) * b.qstride;
                if (clear_basis(d + 1)) return SCD_EHIP;
                // w = St^T N(v_d): the operator applied to the unscaled v_d.
                a.no_x0 = 1;
                a.check = 0;
                a.lc_sweep = cone ? radius_u + 1 + d : -1;
                SCD_HIP(t64.mark(st), "event record");
                SCD_HIP(launch_sweep_f64(g, a, St, S, src_blk, v, w, partial, st),
                        "matvec launch");
                SCD_HIP(t64.mark(st), "event record");
                a.no_x0 = 0;
                stats->fp64_sweeps++;
                stats->sweep_launches++;
                stats->gemm_flops += sweep_flops(cone ? radius_u + 2 + d : 1 << 20, cps);
                const int k = d + 1;
                GsPass q = p;
                q.k = k;
                q.w = w;
                q.radius = cone ? radius_u + 2 + d : -1;   // w reaches one hop beyond v_d
                q.wsig = b.sig + (size_t)d * b.ldx;     // T q_d = sig_d T v_d
                q.pdot = b.pa;
                if (gs(GS_DOTS, q, k + 1)) return SCD_EHIP;          // h1
                q.coef = b.pa;
                q.coef_parts = b.nch;
                q.coef_pstride = pstride;
                q.pdot = b.pb;
                if (gs(GS_PROJ_DOTS, q, k + 1)) return SCD_EHIP;     // h2
                q.coef2 = b.pb;
                if (gs(GS_UPDATE_NORM, q, k + 2)) return SCD_EHIP;   // v_{d+1}, |v_{d+1}|
                ga.d = d;
                SCD_HIP(ts.mark(st), "event record");
                SCD_HIP(launch_givens(ga, st), "Givens launch");
                SCD_HIP(ts.mark(st), "event record");
                ++n;
                if (reduce(r, ngw)) return SCD_EHIP;
                if (r[2] != 0.0 || !std::isfinite(r[0])) {
                    code = fail(SCD_ENAN, "NaN or Inf in the GMRES residual at step %d", n);
                    break;
                }
                e = r[0];
                if (e <= tol || n >= max_iter || d == restart - 1) {
                    // u += sum_i y_i q_i over the k basis vectors of this cycle.
                    SCD_HIP(ts.mark(st), "event record");
                    SCD_HIP(launch_gmres_solve(b.R, b.gv, b.y, k, b.ldx, st), "solve launch");
                    SCD_HIP(ts.mark(st), "event record");
                    GsPass uq = p;
                    uq.k = k;
                    uq.w = b.u;
                    uq.radius = cone ? radius_u + 1 + d : -1;
                    uq.coef = b.y;
                    uq.coef_parts = 1;
                    uq.coef_pstride = 0;
                    if (gs(GS_UPDATE, uq, k + 2)) return SCD_EHIP;
                    radius_u += 1 + d;
                    break;
                }
            }
            // Back to the top: convergence (and the reported error) is decided on
            // the residual recomputed in FP64 from u, not on the rotated estimate.
            if (code == SCD_ENAN) break;
        }
        double tail[3];
        if (reduce(tail, ngw)) return SCD_EHIP;     // drains the last timings
        res->X = b.u;
        res->sweeps = n;
        res->err = e;
        res->rho = (n > 0 && e0 > 0.0 && e > 0.0) ? std::pow(e / e0, 1.0 / n) : 0.0;
        return code;
    }
};

}  // namespace

extern "C" {

const char* scd_last_error(void) { return g_last_error.c_str(); }

int scd_workspace_bytes(const scd_problem* p, int32_t n_src, int32_t block_sites, int32_t prec,
                        size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes) return fail(SCD_EINVAL, "bytes is NULL");
    if (n_src < 1 || n_src > g.n_r) return fail(SCD_EINVAL, "n_src must be in [1, N_r]");
    if (block_sites < 1) return fail(SCD_EINVAL, "block_sites must be >= 1");
    if (prec != SCD_PREC_FP64 && prec != SCD_PREC_FP32 && prec != SCD_PREC_BF16X3)
        return fail(SCD_EINVAL, "unsupported precision %d", prec);
    *bytes = layout(g, n_src, block_sites, prec).total;
    g_last_error.clear();
    return SCD_OK;
}

int sigma_build(const scd_problem* p, const double* V, const double* U, void* S, void* stream) {
    Geom g;
    int rc = check_problem(p, 1024, &g);
    if (rc) return rc;
    if (g.n_real > 512) return fail(SCD_EINVAL, "at most 512 real-time points");
    if (!V || !U || !S) return fail(SCD_EINVAL, "V, U and S must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    SCD_HIP(launch_sigma_build(g, V, U, (double2*)S, st), "sigma_build launch");
    g_last_error.clear();
    return SCD_OK;
}

int local_observables(const scd_problem* p, const void* G_loc, const void* G_nn, const double* J,
                      int32_t n_src, double* n_out, double* ekin_out, void* stream) {
    Geom g;
    int rc = check_problem(p, 1 << 20, &g);
    if (rc) return rc;
    if (n_src < 1) return fail(SCD_EINVAL, "n_src must be >= 1");
    if (!G_loc || !n_out) return fail(SCD_EINVAL, "G_loc and n_out must be non-NULL");
    if (ekin_out && (!G_nn || !J)) return fail(SCD_EINVAL, "ekin_out needs G_nn and J");
    hipStream_t st = (hipStream_t)stream;
    SCD_HIP(launch_observables(g, (const double2*)G_loc, (const double2*)G_nn, J, n_src, n_out,
                               ekin_out, st),
            "local_observables launch");
    g_last_error.clear();
    return SCD_OK;
}

namespace {

// Requested sources of a point-group-reduced solve: the representatives to
// solve, and per requested source (sorted by its representative's position)
// the position within its column block, the group element and the slot map.
struct SymPlan {
    SymGroup grp;
    std::vector<int32_t> reps, req, req_lr, req_g, req_slot, req_pos;
    size_t off_perm = 0, off_perm_inv = 0, off_req = 0, off_lr = 0, off_g = 0, off_slot = 0,
           off_check = 0, total = 0;
};

constexpr int kSymCheckParts = 256;

int sym_plan(const Geom& g, const int32_t* src, int n_src, int block_sites, size_t base,
             SymPlan* P) {
    P->grp = lattice_group(g);
    std::vector<int> pos(g.n_r, -1);
    for (int s = 0; s < n_src; ++s) {
        const int r = P->grp.rep[src[s]];
        if (pos[r] < 0) {
            pos[r] = (int)P->reps.size();
            P->reps.push_back(r);
        }
    }
    const int bs_max = std::min(block_sites, (int)P->reps.size());
    std::vector<int> order(n_src);
    for (int s = 0; s < n_src; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return pos[P->grp.rep[src[a]]] < pos[P->grp.rep[src[b]]];
    });
    for (int s : order) {
        const int rp = pos[P->grp.rep[src[s]]];
        P->req.push_back(s);
        P->req_pos.push_back(rp);
        P->req_lr.push_back(rp % bs_max);
        P->req_g.push_back(P->grp.elem[src[s]]);
        for (int d = 0; d < 4; ++d) {
            const int q = sym_slot(P->grp, g, src[s], d);
            if (q == -2)
                return fail(SCD_EINVAL, "the lattice point group does not map neighbours of "
                                        "site %d to neighbours", src[s]);
            P->req_slot.push_back(q);
        }
    }
    size_t off = base;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t tab = (size_t)P->grp.n_el * g.n_r * sizeof(int32_t);
    P->off_perm = take(tab);
    P->off_perm_inv = take(tab);
    P->off_req = take((size_t)n_src * sizeof(int32_t));
    P->off_lr = take((size_t)n_src * sizeof(int32_t));
    P->off_g = take((size_t)n_src * sizeof(int32_t));
    P->off_slot = take((size_t)n_src * 4 * sizeof(int32_t));
    P->off_check = take(kSymCheckParts * sizeof(double));
    P->total = off;
    return SCD_OK;
}

// dyson_iterate and dyson_iterate_sym: the sweeps over the column blocks of
// `src` (sym: of the orbit representatives of `src`).
int iterate_impl(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                 int32_t n_src, int32_t block_sites, int32_t prec, double tol, int32_t max_iter,
                 void* G_cols, void* G_loc, void* G_nn, void* ws, size_t ws_bytes,
                 scd_stats* st_out, void* stream, bool sym, int max_radius = -1) {
    const auto t_start = std::chrono::steady_clock::now();
    scd_stats stats;
    std::memset(&stats, 0, sizeof stats);
    auto finish = [&](int code) {
        stats.status = code;
        stats.seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (st_out) *st_out = stats;
        return code;
    };

    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return finish(rc);
    if (!S || !J || !src || !G_loc || !ws)
        return finish(fail(SCD_EINVAL, "S, J, src, G_loc and ws must be non-NULL"));
    if (n_src < 1 || n_src > g.n_r) return finish(fail(SCD_EINVAL, "n_src must be in [1, N_r]"));
    if (block_sites < 1) return finish(fail(SCD_EINVAL, "block_sites must be >= 1"));
    if (prec != SCD_PREC_FP64 && prec != SCD_PREC_FP32 && prec != SCD_PREC_BF16X3)
        return finish(fail(SCD_EINVAL, "unsupported precision %d", prec));
    if (!(tol > 0.0) || !std::isfinite(tol)) return finish(fail(SCD_EINVAL, "tol must be > 0"));
    if (max_iter < 1) return finish(fail(SCD_EINVAL, "max_iter must be >= 1"));
    for (int s = 0; s < n_src; ++s)
        if (src[s] < 0 || src[s] >= g.n_r)
            return finish(fail(SCD_EINVAL, "src[%d] = %d outside [0, %d)", s, src[s], g.n_r));
    if (max_radius >= 0 && prec != SCD_PREC_FP64)
        return finish(fail(SCD_EINVAL, "truncation is implemented for SCD_PREC_FP64 only"));
    SymPlan plan;
    const int32_t* solve_src = src;
    int n_solve = n_src;
    if (sym) {
        // Layout of the representatives first, then the symmetry tables after it.
        SymPlan probe;
        rc = sym_plan(g, src, n_src, block_sites, 0, &probe);
        if (rc) return finish(rc);
        const Layout L0 = layout(g, (int)probe.reps.size(), block_sites, prec);
        rc = sym_plan(g, src, n_src, block_sites, L0.total, &plan);
        if (rc) return finish(rc);
        solve_src = plan.reps.data();
        n_solve = (int)plan.reps.size();
    }
    const Layout L = layout(g, n_solve, block_sites, prec);
    const size_t need = sym ? plan.total : L.total;
    if (ws_bytes < need)
        return finish(fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need));

    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    if (sym) {
        // S must be invariant under the group (checked on the generators).
        int* perm_dev = (int*)(base + plan.off_perm);
        const size_t tab = (size_t)plan.grp.n_el * g.n_r * sizeof(int32_t);
        SCD_HIP(hipMemcpyAsync(perm_dev, plan.grp.perm.data(), tab, hipMemcpyHostToDevice, st),
                "copy group");
        SCD_HIP(hipMemcpyAsync(base + plan.off_perm_inv, plan.grp.perm_inv.data(), tab,
                               hipMemcpyHostToDevice, st),
                "copy group");
        const size_t nq = plan.req.size() * sizeof(int32_t);
        SCD_HIP(hipMemcpyAsync(base + plan.off_req, plan.req.data(), nq, hipMemcpyHostToDevice, st),
                "copy plan");
        SCD_HIP(hipMemcpyAsync(base + plan.off_lr, plan.req_lr.data(), nq, hipMemcpyHostToDevice,
                               st),
                "copy plan");
        SCD_HIP(hipMemcpyAsync(base + plan.off_g, plan.req_g.data(), nq, hipMemcpyHostToDevice, st),
                "copy plan");
        SCD_HIP(hipMemcpyAsync(base + plan.off_slot, plan.req_slot.data(), 4 * nq,
                               hipMemcpyHostToDevice, st),
                "copy plan");
        double worst = 0.0;
        const int gens[3] = {1, 2, 4};
        for (int e : gens) {
            if (e >= plan.grp.n_el) continue;
            double part[kSymCheckParts];
            double* part_dev = (double*)(base + plan.off_check);
            SCD_HIP(launch_sym_check((const double2*)S, perm_dev + (size_t)e * g.n_r, g, part_dev,
                                     kSymCheckParts, st),
                    "symmetry check launch");
            SCD_HIP(hipMemcpyAsync(part, part_dev, sizeof part, hipMemcpyDeviceToHost, st),
                    "copy check");
            SCD_HIP(hipStreamSynchronize(st), "check sync");
            for (double v : part) worst = (v > worst || v != v) ? v : worst;
        }
        if (!(worst <= 1e-12))
            return finish(fail(SCD_EINVAL,
                                "S is not invariant under the lattice point group "
                                "(max |S_i - S_g(i)| = %g)",
                                worst));
    }
    Solver sv;
    sv.g = g;
    sv.st = st;
    sv.stats = &stats;
    sv.St = (double2*)(base + L.off_st);
    sv.St32 = prec != SCD_PREC_FP64 ? (void*)(base + L.off_st32) : nullptr;
    sv.bf3 = prec == SCD_PREC_BF16X3;
    sv.S = (const double2*)S;
    sv.partial = (double*)(base + L.off_partial);
    sv.slot = (unsigned long long*)(base + L.off_slot);
    sv.nwg = L.nwg;
    sv.trunc = max_radius;
    int* src_dev = (int*)(base + L.off_src);

    SCD_HIP(hipMemcpyAsync(src_dev, solve_src, (size_t)n_solve * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy src");
    const bool bipartite = lattice_bipartite(g);
    int n_even = 0;
    const std::vector<int32_t> order = colour_order(g, site_group(g), bipartite, &n_even);
    int* order_dev = (int*)(base + L.off_order);
    SCD_HIP(hipMemcpyAsync(order_dev, order.data(), (size_t)g.n_r * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy site order");
    sv.all_sites = order_dev;
    if (bipartite) {
        sv.colour_sites[0] = order_dev;
        sv.colour_sites[1] = order_dev + n_even;
        sv.n_colour[0] = n_even;
        sv.n_colour[1] = g.n_r - n_even;
    }
    SCD_HIP(launch_scale_transpose(g, (const double2*)S, J, sv.St, 0, st), "scale_transpose launch");
    if (sv.bf3)
        SCD_HIP(launch_bf3_operand(g, sv.St, sv.St32, st), "BF16x3 operand launch");
    else if (sv.St32)
        SCD_HIP(launch_to_f32(sv.St, sv.St32, (size_t)g.n_r * g.mp * g.mp, st), "St32 launch");
    SCD_HIP(hipStreamSynchronize(st), "setup sync");

    const int bs_max = block_sites < n_solve ? block_sites : n_solve;
    double worst_err = 0.0, worst_rho = 0.0;
    int final_code = SCD_OK;
    for (int blk_start = 0; blk_start < n_solve; blk_start += bs_max) {
        const int bs = (n_solve - blk_start) < bs_max ? (n_solve - blk_start) : bs_max;
        const int* src_blk = src_dev + blk_start;
        SweepArgs a;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.periodic = g.periodic;
        a.n_r = g.n_r;
        a.n_t = g.n_t;
        a.ldx = L.ldx;
        a.ntn = L.ntn;
        a.bs = bs;
        a.lc_sweep = 0;
        a.group = site_group(g);
        a.x0_kind = X0_BLOCK;
        a.x0_fixed = 0;
        a.max_radius = max_radius;
        a.sites = nullptr;
        a.n_sites = g.n_r;
        a.part_off = 0;
        a.check = 1;
        sv.pair_counts(solve_src + blk_start, bs);
        double2* X = (double2*)(base + L.off_x0);
        double2* Xn = L.off_x1 ? (double2*)(base + L.off_x1) : nullptr;
        SCD_HIP(launch_init_block(g, (const double2*)S, src_blk, bs, L.ldx, X0_BLOCK, 0, X, Xn, st),
                "init_block launch");
        BlockResult res;
        int code;
        if (prec == SCD_PREC_FP64) {
            code = sv.solve_fp64(a, src_blk, X, Xn, tol, max_iter, &res);
        } else {
            code = sv.solve_mixed(a, src_blk, X, base + L.off_r32, base + L.off_d0,
                                  L.off_d1 ? base + L.off_d1 : nullptr, tol, max_iter, &res);
        }
        if (code == SCD_EHIP) return finish(code);
        if (code == SCD_ENOTCONV)
            fail(SCD_ENOTCONV, "block at source %d not converged after %d sweeps (e=%g)", blk_start,
                 max_iter, res.err);
        stats.n_blocks++;
        stats.sweeps_total += res.sweeps;
        if (res.sweeps > stats.sweeps_max) stats.sweeps_max = res.sweeps;
        worst_err = res.err > worst_err ? res.err : worst_err;
        worst_rho = res.rho > worst_rho ? res.rho : worst_rho;
        if (sym) {
            // Every requested source whose representative is in this block.
            int q0 = 0;
            while (q0 < n_src && plan.req_pos[q0] < blk_start) ++q0;
            int q1 = q0;
            while (q1 < n_src && plan.req_pos[q1] < blk_start + bs) ++q1;
            SCD_HIP(launch_extract_sym(g, res.X, L.ldx, src_blk, (int*)(base + plan.off_req) + q0,
                                       (int*)(base + plan.off_lr) + q0,
                                       (int*)(base + plan.off_g) + q0,
                                       (int*)(base + plan.off_slot) + 4 * q0,
                                       (int*)(base + plan.off_perm_inv), q1 - q0, n_src,
                                       (double2*)G_cols, (double2*)G_loc, (double2*)G_nn, st),
                    "extract launch");
        } else {
            SCD_HIP(launch_extract(g, res.X, L.ldx, src_blk, bs, blk_start, n_src,
                                   (double2*)G_cols, (double2*)G_loc, (double2*)G_nn, st),
                    "extract launch");
        }
        if (code != SCD_OK) {
            final_code = code;
            break;
        }
    }
    SCD_HIP(hipStreamSynchronize(st), "final sync");
    stats.final_err = worst_err;
    stats.rho_est = worst_rho;
    if (final_code == SCD_OK) g_last_error.clear();
    return finish(final_code);
}

}  // namespace

namespace {

struct S2Layout {
    size_t off_k, off_part, off_m, off_aug, off_flag, total;
};

S2Layout s2_layout(const Geom& g) {
    S2Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    const size_t blocks = (size_t)g.n_r * g.n_t * g.n_t * sizeof(double2);
    L.off_k = take(blocks);
    L.off_part = take(blocks);
    L.off_m = take(blocks);
    L.off_aug = take(2 * blocks);
    L.off_flag = take(sizeof(int));
    L.total = off;
    return L;
}

}  // namespace

int scd_sigma2_workspace_bytes(const scd_problem* p, size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes) return fail(SCD_EINVAL, "bytes is NULL");
    *bytes = s2_layout(g).total;
    g_last_error.clear();
    return SCD_OK;
}

int sigma2_build(const scd_problem* p, const double* V, const double* U, const double* J,
                 const void* S, const void* G_loc_all, void* sig_out, void* ws, size_t ws_bytes,
                 void* stream) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!V || !U || !J || !S || !G_loc_all || !sig_out || !ws)
        return fail(SCD_EINVAL, "V, U, J, S, G_loc_all, sig_out and ws must be non-NULL");
    const S2Layout L = s2_layout(g);
    if (ws_bytes < L.total)
        return fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    SCD_HIP(launch_sigma2(g, V, U, J, (const double2*)S, (const double2*)G_loc_all,
                          (double2*)(base + L.off_k), (double2*)(base + L.off_part),
                          (double2*)(base + L.off_m), (double2*)sig_out, st),
            "sigma2 launch");
    g_last_error.clear();
    return SCD_OK;
}

int sigma2_dress(const scd_problem* p, const void* S, const void* sig, void* S_out, void* ws,
                 size_t ws_bytes, void* stream) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!S || !sig || !S_out || !ws) return fail(SCD_EINVAL, "S, sig, S_out and ws must be non-NULL");
    if (S_out == S) return fail(SCD_EINVAL, "S_out must not alias S");
    const S2Layout L = s2_layout(g);
    if (ws_bytes < L.total)
        return fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    int* flag = (int*)(base + L.off_flag);
    SCD_HIP(hipMemsetAsync(flag, 0, sizeof(int), st), "flag clear");
    SCD_HIP(launch_dress(g, (const double2*)S, (const double2*)sig, (double2*)(base + L.off_aug),
                         (double2*)S_out, flag, st),
            "dress launch");
    int h = 0;
    SCD_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, st), "flag copy");
    SCD_HIP(hipStreamSynchronize(st), "dress sync");
    if (h) return fail(SCD_ENAN, "S - Sigma~ is singular on some site");
    g_last_error.clear();
    return SCD_OK;
}

int dyson_selfconsistent(const scd_problem* p, const double* V, const double* U, const double* J,
                         double lam, double delta_sc, int32_t max_sc, int32_t block_sites,
                         int32_t prec, double tol, int32_t max_iter, void* S_out, void* sig_out,
                         void* G_loc, void* G_nn, void* ws, size_t ws_bytes, int32_t* sc_iter,
                         double* sc_norm, scd_stats* st_out, void* stream) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!V || !U || !J || !S_out || !sig_out || !G_loc || !ws)
        return fail(SCD_EINVAL, "V, U, J, S_out, sig_out, G_loc and ws must be non-NULL");
    if (!(lam > 0.0 && lam <= 1.0)) return fail(SCD_EINVAL, "lam must be in (0, 1]");
    if (!(delta_sc > 0.0)) return fail(SCD_EINVAL, "delta_sc must be > 0");
    if (max_sc < 1) return fail(SCD_EINVAL, "max_sc must be >= 1");
    size_t need = 0;
    size_t dyson_bytes = 0, s2_bytes = 0;
    rc = scd_workspace_bytes(p, g.n_r, block_sites, prec, &dyson_bytes);
    if (rc) return rc;
    rc = scd_sigma2_workspace_bytes(p, &s2_bytes);
    if (rc) return rc;
    const size_t blocks = align256((size_t)g.n_r * g.n_t * g.n_t * sizeof(double2));
    constexpr int kParts = 1024;
    const size_t off_dressed = 0, off_new = blocks, off_s2 = 2 * blocks,
                 off_dyson = off_s2 + align256(s2_bytes),
                 off_part = off_dyson + align256(dyson_bytes);
    need = off_part + align256(2 * kParts * sizeof(double));
    if (ws_bytes < need) return fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    double2* S = (double2*)S_out;
    double2* sig = (double2*)sig_out;
    double2* dressed = (double2*)(base + off_dressed);
    double2* fresh = (double2*)(base + off_new);
    void* ws2 = base + off_s2;
    void* wsd = base + off_dyson;
    double* part = (double*)(base + off_part);
    const size_t n_el = (size_t)g.n_r * g.n_t * g.n_t;
    std::vector<int32_t> every(g.n_r);
    for (int i = 0; i < g.n_r; ++i) every[i] = i;
    scd_stats total;
    std::memset(&total, 0, sizeof total);
    auto accumulate = [&](const scd_stats& s) {
        total.n_blocks += s.n_blocks;
        total.sweeps_total += s.sweeps_total;
        total.sweeps_max = std::max(total.sweeps_max, s.sweeps_max);
        total.fp64_sweeps += s.fp64_sweeps;
        total.lowp_sweeps += s.lowp_sweeps;
        total.final_err = s.final_err;
        total.rho_est = s.rho_est;
        total.gemm_flops += s.gemm_flops;
        total.seconds += s.seconds;
        total.sweep_kernel_seconds += s.sweep_kernel_seconds;
        total.lowp_kernel_seconds += s.lowp_kernel_seconds;
        total.sweep_launches += s.sweep_launches;
        total.lowp_launches += s.lowp_launches;
    };
    rc = sigma_build(p, V, U, S, stream);
    if (rc) return rc;
    SCD_HIP(hipMemsetAsync(sig, 0, n_el * sizeof(double2), st), "clear Sigma~");
    int it = 0;
    double norm = 0.0;
    int code = SCD_ENOTCONV;
    for (it = 1; it <= max_sc; ++it) {
        // G_loc of every site with the current dressed blocks
        rc = sigma2_dress(p, S, sig, dressed, ws2, s2_bytes, stream);
        if (rc) return rc;
        scd_stats s1;
        rc = dyson_iterate(p, dressed, J, every.data(), g.n_r, block_sites, prec, tol, max_iter,
                           nullptr, G_loc, G_nn, wsd, dyson_bytes, &s1, stream);
        accumulate(s1);
        if (rc) return rc;
        rc = sigma2_build(p, V, U, J, S, G_loc, fresh, ws2, s2_bytes, stream);
        if (rc) return rc;
        SCD_HIP(launch_mix(fresh, sig, lam, n_el, part, kParts, st), "mix launch");
        std::vector<double> h(2 * kParts);
        SCD_HIP(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st),
                "copy partials");
        SCD_HIP(hipStreamSynchronize(st), "mix sync");
        double s2 = 0.0, mx = 0.0;
        for (int w = 0; w < kParts; ++w) {
            s2 += h[2 * w];
            mx = (h[2 * w + 1] > mx || h[2 * w + 1] != h[2 * w + 1]) ? h[2 * w + 1] : mx;
        }
        // |Delta|_F / N_bd + |Delta|_max (Sec. III), on Sigma~
        norm = std::sqrt(s2) / (double)n_el + mx;
        if (!std::isfinite(norm)) {
            code = fail(SCD_ENAN, "NaN or Inf in Sigma~ at self-consistency step %d", it);
            break;
        }
        if (norm <= delta_sc) {
            code = SCD_OK;
            break;
        }
    }
    if (code != SCD_ENAN) {
        // the solve with the final (mixed) self-energy
        rc = sigma2_dress(p, S, sig, dressed, ws2, s2_bytes, stream);
        if (rc) return rc;
        scd_stats s1;
        rc = dyson_iterate(p, dressed, J, every.data(), g.n_r, block_sites, prec, tol, max_iter,
                           nullptr, G_loc, G_nn, wsd, dyson_bytes, &s1, stream);
        accumulate(s1);
        if (rc) return rc;
    }
    if (sc_iter) *sc_iter = it > max_sc ? max_sc : it;
    if (sc_norm) *sc_norm = norm;
    total.status = code;
    if (st_out) *st_out = total;
    if (code == SCD_ENOTCONV)
        return fail(SCD_ENOTCONV, "self-consistency not reached after %d steps (norm %g)", max_sc,
                    norm);
    if (code == SCD_OK) g_last_error.clear();
    return code;
}

int scd_selfconsistent_workspace_bytes(const scd_problem* p, int32_t block_sites, int32_t prec,
                                       size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes) return fail(SCD_EINVAL, "bytes is NULL");
    size_t dyson_bytes = 0, s2_bytes = 0;
    rc = scd_workspace_bytes(p, g.n_r, block_sites, prec, &dyson_bytes);
    if (rc) return rc;
    rc = scd_sigma2_workspace_bytes(p, &s2_bytes);
    if (rc) return rc;
    const size_t blocks = align256((size_t)g.n_r * g.n_t * g.n_t * sizeof(double2));
    *bytes = 2 * blocks + align256(s2_bytes) + align256(dyson_bytes) +
             align256(2 * 1024 * sizeof(double));
    g_last_error.clear();
    return SCD_OK;
}

int double_occupancy(const scd_problem* p, const void* G_loc, const void* G_nn, const double* J,
                     const double* V, const double* U, const int32_t* src, int32_t n_src,
                     double* d_out, double* frac_out, void* stream) {
    Geom g;
    int rc = check_problem(p, 1 << 20, &g);
    if (rc) return rc;
    if (n_src < 1) return fail(SCD_EINVAL, "n_src must be >= 1");
    if (g.n_real < 2) return fail(SCD_EINVAL, "the time derivative needs n_real >= 2");
    if (!G_loc || !G_nn || !J || !V || !U || !src || !d_out)
        return fail(SCD_EINVAL, "G_loc, G_nn, J, V, U, src and d_out must be non-NULL");
    hipStream_t st = (hipStream_t)stream;
    SCD_HIP(launch_docc(g, (const double2*)G_loc, (const double2*)G_nn, J, V, U, src, n_src, d_out,
                        frac_out, st),
            "double_occupancy launch");
    g_last_error.clear();
    return SCD_OK;
}

int scd_extrapolate_dt(const double* dts, int32_t n_dt, const double* values, int32_t n,
                       double* out) {
    if (!dts || !values || !out) return fail(SCD_EINVAL, "dts, values and out must be non-NULL");
    if (n_dt != 2 && n_dt != 3) return fail(SCD_EINVAL, "two or three step sizes");
    if (n < 0) return fail(SCD_EINVAL, "n must be >= 0");
    for (int k = 0; k < n_dt; ++k)
        for (int j = 0; j < k; ++j)
            if (!(dts[k] != dts[j])) return fail(SCD_EINVAL, "step sizes must differ");
    // Lagrange weights of the interpolating polynomial at dt = 0.
    double w[3];
    for (int k = 0; k < n_dt; ++k) {
        w[k] = 1.0;
        for (int j = 0; j < n_dt; ++j)
            if (j != k) w[k] *= (0.0 - dts[j]) / (dts[k] - dts[j]);
    }
    for (int i = 0; i < n; ++i) {
        double v = 0.0;
        for (int k = 0; k < n_dt; ++k) v += w[k] * values[(size_t)k * n + i];
        out[i] = v;
    }
    g_last_error.clear();
    return SCD_OK;
}

int dyson_iterate(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                  int32_t n_src, int32_t block_sites, int32_t prec, double tol, int32_t max_iter,
                  void* G_cols, void* G_loc, void* G_nn, void* ws, size_t ws_bytes,
                  scd_stats* st_out, void* stream) {
    return iterate_impl(p, S, J, src, n_src, block_sites, prec, tol, max_iter, G_cols, G_loc, G_nn,
                        ws, ws_bytes, st_out, stream, false);
}

int dyson_iterate_sym(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                      int32_t n_src, int32_t block_sites, int32_t prec, double tol,
                      int32_t max_iter, void* G_cols, void* G_loc, void* G_nn, void* ws,
                      size_t ws_bytes, scd_stats* st_out, void* stream) {
    return iterate_impl(p, S, J, src, n_src, block_sites, prec, tol, max_iter, G_cols, G_loc, G_nn,
                        ws, ws_bytes, st_out, stream, true);
}

int dyson_iterate_trunc(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                        int32_t n_src, int32_t block_sites, int32_t max_radius, double tol,
                        int32_t max_iter, void* G_cols, void* G_loc, void* G_nn, void* ws,
                        size_t ws_bytes, scd_stats* st_out, void* stream) {
    if (max_radius < 0) return fail(SCD_EINVAL, "max_radius must be >= 0");
    return iterate_impl(p, S, J, src, n_src, block_sites, SCD_PREC_FP64, tol, max_iter, G_cols,
                        G_loc, G_nn, ws, ws_bytes, st_out, stream, false, max_radius);
}

int scd_sym_workspace_bytes(const scd_problem* p, const int32_t* src, int32_t n_src,
                            int32_t block_sites, int32_t prec, size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes || !src) return fail(SCD_EINVAL, "src and bytes must be non-NULL");
    if (n_src < 1 || n_src > g.n_r) return fail(SCD_EINVAL, "n_src must be in [1, N_r]");
    if (block_sites < 1) return fail(SCD_EINVAL, "block_sites must be >= 1");
    if (prec != SCD_PREC_FP64 && prec != SCD_PREC_FP32 && prec != SCD_PREC_BF16X3)
        return fail(SCD_EINVAL, "unsupported precision %d", prec);
    for (int s = 0; s < n_src; ++s)
        if (src[s] < 0 || src[s] >= g.n_r)
            return fail(SCD_EINVAL, "src[%d] = %d outside [0, %d)", s, src[s], g.n_r);
    SymPlan probe;
    rc = sym_plan(g, src, n_src, block_sites, 0, &probe);
    if (rc) return rc;
    SymPlan plan;
    rc = sym_plan(g, src, n_src, block_sites,
                  layout(g, (int)probe.reps.size(), block_sites, prec).total, &plan);
    if (rc) return rc;
    *bytes = plan.total;
    g_last_error.clear();
    return SCD_OK;
}

// ---- GMRES -----------------------------------------------------------------

namespace {

struct GmLayout {
    int ldx, ntn, nwg, nch, rows, chunk_rows;
    size_t off_st, off_u, off_q, qstride_bytes, off_pa, off_pb, off_pn, off_sig, off_R, off_cs,
        off_sn, off_g, off_y, off_x0n, off_partial, off_slot, off_src, off_order, total;
};

// Workspace of dyson_gmres: St, the iterate u, restart + 1 basis vectors (each
// an FP64 block iterate), the Gram-Schmidt partials and per-column Hessenberg
// state (O(kMaxBasis^2) complex per column).
GmLayout gm_layout(const Geom& g, int n_src, int block_sites, int restart) {
    GmLayout L;
    const int bs = block_sites < n_src ? block_sites : n_src;
    L.ldx = ((bs * g.n_t + kColsPerWG - 1) / kColsPerWG) * kColsPerWG;
    L.ntn = L.ldx / kColsPerWG;
    L.nwg = g.n_r * L.ntn;
    L.rows = g.n_r * g.mp;
    // Row chunks of whole sites (the passes skip chunks outside the light
    // cone); nch is exactly the number of chunks a pass launches.
    const int spc = (g.n_r + gs_chunks(L.rows, L.ldx) - 1) / gs_chunks(L.rows, L.ldx);
    L.nch = (g.n_r + spc - 1) / spc;
    L.chunk_rows = spc * g.mp;
    const size_t it64 = (size_t)L.rows * L.ldx * sizeof(double2);
    const size_t col = (size_t)L.ldx;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.off_st = take((size_t)g.n_r * g.mp * g.mp * sizeof(double2));
    L.off_u = take(it64);
    L.qstride_bytes = align256(it64);
    L.off_q = take(L.qstride_bytes * (size_t)(restart + 1));
    L.off_pa = take((size_t)L.nch * kMaxBasis * col * sizeof(double2));
    L.off_pb = take((size_t)L.nch * kMaxBasis * col * sizeof(double2));
    L.off_pn = take((size_t)L.nch * col * sizeof(double));
    L.off_sig = take((size_t)(kMaxBasis + 1) * col * sizeof(double));
    L.off_R = take((size_t)kMaxBasis * kMaxBasis * col * sizeof(double2));
    L.off_cs = take((size_t)kMaxBasis * col * sizeof(double));
    L.off_sn = take((size_t)kMaxBasis * col * sizeof(double2));
    L.off_g = take((size_t)(kMaxBasis + 1) * col * sizeof(double2));
    L.off_y = take((size_t)kMaxBasis * col * sizeof(double2));
    L.off_x0n = take(col * sizeof(double));
    const size_t nparts = std::max((size_t)L.nwg, (L.ldx + 255) / (size_t)256);
    L.off_partial = take(nparts * 3 * sizeof(double));
    L.off_slot = take(4 * sizeof(unsigned long long));
    L.off_src = take((size_t)n_src * sizeof(int32_t));
    L.off_order = take((size_t)g.n_r * sizeof(int32_t));
    L.total = off;
    return L;
}

}  // namespace

int scd_gmres_workspace_bytes(const scd_problem* p, int32_t n_src, int32_t block_sites,
                              int32_t restart, size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes) return fail(SCD_EINVAL, "bytes is NULL");
    if (n_src < 1 || n_src > g.n_r) return fail(SCD_EINVAL, "n_src must be in [1, N_r]");
    if (block_sites < 1) return fail(SCD_EINVAL, "block_sites must be >= 1");
    if (restart < 1 || restart > kMaxBasis)
        return fail(SCD_EINVAL, "restart must be in [1, %d]", kMaxBasis);
    *bytes = gm_layout(g, n_src, block_sites, restart).total;
    g_last_error.clear();
    return SCD_OK;
}

int dyson_gmres(const scd_problem* p, const void* S, const double* J, const int32_t* src,
                int32_t n_src, int32_t block_sites, int32_t restart, double tol, int32_t max_iter,
                void* G_cols, void* G_loc, void* G_nn, void* ws, size_t ws_bytes,
                scd_stats* st_out, void* stream) {
    const auto t_start = std::chrono::steady_clock::now();
    scd_stats stats;
    std::memset(&stats, 0, sizeof stats);
    auto finish = [&](int code) {
        stats.status = code;
        stats.seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (st_out) *st_out = stats;
        return code;
    };
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return finish(rc);
    if (!S || !J || !src || !G_loc || !ws)
        return finish(fail(SCD_EINVAL, "S, J, src, G_loc and ws must be non-NULL"));
    if (n_src < 1 || n_src > g.n_r) return finish(fail(SCD_EINVAL, "n_src must be in [1, N_r]"));
    if (block_sites < 1) return finish(fail(SCD_EINVAL, "block_sites must be >= 1"));
    if (restart < 1 || restart > kMaxBasis)
        return finish(fail(SCD_EINVAL, "restart must be in [1, %d]", kMaxBasis));
    if (!(tol > 0.0) || !std::isfinite(tol)) return finish(fail(SCD_EINVAL, "tol must be > 0"));
    if (max_iter < 1) return finish(fail(SCD_EINVAL, "max_iter must be >= 1"));
    for (int s = 0; s < n_src; ++s)
        if (src[s] < 0 || src[s] >= g.n_r)
            return finish(fail(SCD_EINVAL, "src[%d] = %d outside [0, %d)", s, src[s], g.n_r));
    const GmLayout L = gm_layout(g, n_src, block_sites, restart);
    if (ws_bytes < L.total)
        return finish(fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total));

    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    Solver sv;
    sv.g = g;
    sv.st = st;
    sv.stats = &stats;
    sv.St = (double2*)(base + L.off_st);
    sv.St32 = nullptr;
    sv.S = (const double2*)S;
    sv.partial = (double*)(base + L.off_partial);
    sv.slot = (unsigned long long*)(base + L.off_slot);
    sv.nwg = L.nwg;
    int* src_dev = (int*)(base + L.off_src);
    SCD_HIP(hipMemcpyAsync(src_dev, src, (size_t)n_src * sizeof(int32_t), hipMemcpyHostToDevice, st),
            "copy src");
    int n_even = 0;
    const std::vector<int32_t> order = colour_order(g, site_group(g), lattice_bipartite(g), &n_even);
    int* order_dev = (int*)(base + L.off_order);
    SCD_HIP(hipMemcpyAsync(order_dev, order.data(), (size_t)g.n_r * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy site order");
    sv.all_sites = order_dev;     // every launch is Jacobi-style (all sites)
    SCD_HIP(launch_scale_transpose(g, (const double2*)S, J, sv.St, 0, st), "scale_transpose launch");
    SCD_HIP(hipStreamSynchronize(st), "setup sync");

    GmBufs b;
    b.u = (double2*)(base + L.off_u);
    b.Q = (double2*)(base + L.off_q);
    b.qstride = L.qstride_bytes / sizeof(double2);
    b.pa = (double2*)(base + L.off_pa);
    b.pb = (double2*)(base + L.off_pb);
    b.pn = (double*)(base + L.off_pn);
    b.sig = (double*)(base + L.off_sig);
    b.R = (double2*)(base + L.off_R);
    b.cs = (double*)(base + L.off_cs);
    b.sn = (double2*)(base + L.off_sn);
    b.gv = (double2*)(base + L.off_g);
    b.y = (double2*)(base + L.off_y);
    b.x0n = (double*)(base + L.off_x0n);
    b.rows = L.rows;
    b.ldx = L.ldx;
    b.nch = L.nch;
    b.chunk_rows = L.chunk_rows;

    const int bs_max = block_sites < n_src ? block_sites : n_src;
    double worst_err = 0.0, worst_rho = 0.0;
    int final_code = SCD_OK;
    for (int blk_start = 0; blk_start < n_src; blk_start += bs_max) {
        const int bs = (n_src - blk_start) < bs_max ? (n_src - blk_start) : bs_max;
        const int* src_blk = src_dev + blk_start;
        SweepArgs a;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.periodic = g.periodic;
        a.n_r = g.n_r;
        a.n_t = g.n_t;
        a.ldx = L.ldx;
        a.ntn = L.ntn;
        a.bs = bs;
        a.lc_sweep = 0;
        a.group = site_group(g);
        a.x0_kind = X0_BLOCK;
        a.x0_fixed = 0;
        a.sites = nullptr;
        a.n_sites = g.n_r;
        a.part_off = 0;
        a.check = 1;
        sv.pair_counts(src + blk_start, bs);
        SCD_HIP(launch_init_block(g, (const double2*)S, src_blk, bs, L.ldx, X0_BLOCK, 0, b.u,
                                  nullptr, st),
                "init_block launch");
        BlockResult res;
        const int code = sv.solve_gmres(a, src_blk, src + blk_start, b, restart, tol, max_iter,
                                        &res);
        if (code == SCD_EHIP) return finish(code);
        if (code == SCD_ENOTCONV)
            fail(SCD_ENOTCONV, "block at source %d not converged after %d GMRES steps (e=%g)",
                 blk_start, max_iter, res.err);
        stats.n_blocks++;
        stats.sweeps_total += res.sweeps;
        if (res.sweeps > stats.sweeps_max) stats.sweeps_max = res.sweeps;
        worst_err = std::max(worst_err, res.err);
        worst_rho = std::max(worst_rho, res.rho);
        SCD_HIP(launch_extract(g, res.X, L.ldx, src_blk, bs, blk_start, n_src, (double2*)G_cols,
                               (double2*)G_loc, (double2*)G_nn, st),
                "extract launch");
        if (code != SCD_OK) {
            final_code = code;
            break;
        }
    }
    SCD_HIP(hipStreamSynchronize(st), "final sync");
    stats.final_err = worst_err;
    stats.rho_est = worst_rho;
    if (final_code == SCD_OK) g_last_error.clear();
    return finish(final_code);
}

// ---- adjoint ---------------------------------------------------------------

namespace {

struct AdjLayout {
    int ldx, ntn, nwg;
    size_t off_st, off_stt, off_st32, off_stt32, off_xg, off_xh, off_x1, off_r32, off_d0, off_d1,
        off_lam, off_rsum, off_csum, off_bz, off_djc, off_partial, off_slot, off_src, off_order,
        total;
};

AdjLayout adj_layout(const Geom& g, int prec) {
    AdjLayout L;
    L.ldx = ((g.n_r + kColsPerWG - 1) / kColsPerWG) * kColsPerWG;
    L.ntn = L.ldx / kColsPerWG;
    L.nwg = g.n_r * L.ntn;
    const size_t op64 = align256((size_t)g.n_r * g.mp * g.mp * sizeof(double2));
    const size_t op32 = align256(prec == SCD_PREC_BF16X3
                                     ? bf3_operand_bytes(g)
                                     : (size_t)g.n_r * g.mp * g.mp * sizeof(float2));
    const size_t it64 = align256((size_t)g.n_r * g.mp * L.ldx * sizeof(double2));
    const size_t it32 = align256((size_t)g.n_r * g.mp * L.ldx * sizeof(float2));
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += align256(bytes);
        return o;
    };
    L.off_st = take(op64);
    L.off_stt = take(op64);
    L.off_xg = take(it64);
    L.off_xh = take(it64);
    const bool rb = lattice_bipartite(g);
    L.off_st32 = L.off_stt32 = L.off_x1 = L.off_r32 = L.off_d0 = L.off_d1 = 0;
    if (prec == SCD_PREC_FP64) {
        if (!rb) L.off_x1 = take(it64);
    } else {
        L.off_st32 = take(op32);
        L.off_stt32 = take(op32);
        L.off_r32 = take(it32);
        L.off_d0 = take(it32);
        if (!rb) L.off_d1 = take(it32);
    }
    L.off_lam = take((size_t)g.n_r * g.n_t * g.n_t * sizeof(double2));
    L.off_rsum = take((size_t)g.n_r * g.n_t * sizeof(double2));
    L.off_csum = take((size_t)g.n_r * g.n_t * sizeof(double2));
    L.off_bz = take((size_t)g.n_r * sizeof(double));
    L.off_djc = take((size_t)g.n_t * sizeof(double));
    L.off_partial = take((size_t)L.nwg * 3 * sizeof(double));
    L.off_slot = take(4 * sizeof(unsigned long long));
    L.off_src = take((size_t)g.n_r * sizeof(int32_t));
    L.off_order = take((size_t)g.n_r * sizeof(int32_t));
    L.total = off;
    return L;
}

}  // namespace

int scd_adjoint_workspace_bytes(const scd_problem* p, int32_t prec, size_t* bytes) {
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return rc;
    if (!bytes) return fail(SCD_EINVAL, "bytes is NULL");
    if (prec != SCD_PREC_FP64 && prec != SCD_PREC_FP32 && prec != SCD_PREC_BF16X3)
        return fail(SCD_EINVAL, "unsupported precision %d", prec);
    *bytes = adj_layout(g, prec).total;
    g_last_error.clear();
    return SCD_OK;
}

int dyson_adjoint(const scd_problem* p, const void* S, const double* V, const double* U,
                  const double* J, const double* w_loss, int32_t t_index, int32_t prec, double tol,
                  int32_t max_iter, double* n_te, double* loss, double* dV, double* dU, double* dJ,
                  void* ws, size_t ws_bytes, scd_stats* st_out, void* stream) {
    const auto t_start = std::chrono::steady_clock::now();
    scd_stats stats;
    std::memset(&stats, 0, sizeof stats);
    auto finish = [&](int code) {
        stats.status = code;
        stats.seconds =
            std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        if (st_out) *st_out = stats;
        return code;
    };
    Geom g;
    int rc = check_problem(p, kMaxNt, &g);
    if (rc) return finish(rc);
    if (g.n_r > 65535) return finish(fail(SCD_EINVAL, "too many sites"));
    const bool grads = dV || dU || dJ;
    if (grads && !(dV && dU && dJ))
        return finish(fail(SCD_EINVAL, "dV, dU and dJ must be given together"));
    if (!S || !J || !ws) return finish(fail(SCD_EINVAL, "S, J and ws must be non-NULL"));
    if (grads && (!V || !U)) return finish(fail(SCD_EINVAL, "gradients need V and U"));
    if ((grads || loss) && !w_loss) return finish(fail(SCD_EINVAL, "the loss needs w_loss"));
    if (!grads && !loss && !n_te) return finish(fail(SCD_EINVAL, "nothing to compute"));
    if (t_index < 0 || t_index >= g.n_real)
        return finish(fail(SCD_EINVAL, "t_index must be in [0, n_real)"));
    if (prec != SCD_PREC_FP64 && prec != SCD_PREC_FP32 && prec != SCD_PREC_BF16X3)
        return finish(fail(SCD_EINVAL, "unsupported precision %d", prec));
    if (!(tol > 0.0) || !std::isfinite(tol)) return finish(fail(SCD_EINVAL, "tol must be > 0"));
    if (max_iter < 1) return finish(fail(SCD_EINVAL, "max_iter must be >= 1"));
    const AdjLayout L = adj_layout(g, prec);
    if (ws_bytes < L.total)
        return finish(fail(SCD_ENOMEM, "workspace has %zu bytes, %zu needed", ws_bytes, L.total));

    hipStream_t st = (hipStream_t)stream;
    char* base = (char*)ws;
    std::vector<int32_t> ident(g.n_r);
    for (int i = 0; i < g.n_r; ++i) ident[i] = i;
    int* src_dev = (int*)(base + L.off_src);
    SCD_HIP(hipMemcpyAsync(src_dev, ident.data(), (size_t)g.n_r * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy src");
    double2* St = (double2*)(base + L.off_st);
    double2* StT = (double2*)(base + L.off_stt);
    SCD_HIP(launch_scale_transpose(g, (const double2*)S, J, St, 0, st), "operand launch");
    if (grads) SCD_HIP(launch_scale_transpose(g, (const double2*)S, J, StT, 1, st), "operand launch");
    if (prec != SCD_PREC_FP64) {
        const size_t n_op = (size_t)g.n_r * g.mp * g.mp;
        if (prec == SCD_PREC_BF16X3) {
            SCD_HIP(launch_bf3_operand(g, St, base + L.off_st32, st), "BF16x3 operand launch");
            if (grads)
                SCD_HIP(launch_bf3_operand(g, StT, base + L.off_stt32, st),
                        "BF16x3 operand launch");
        } else {
            SCD_HIP(launch_to_f32(St, base + L.off_st32, n_op, st), "St32 launch");
            if (grads) SCD_HIP(launch_to_f32(StT, base + L.off_stt32, n_op, st), "St32 launch");
        }
    }
    SCD_HIP(hipStreamSynchronize(st), "setup sync");

    Solver sv;
    sv.g = g;
    sv.st = st;
    sv.stats = &stats;
    sv.S = (const double2*)S;
    sv.partial = (double*)(base + L.off_partial);
    sv.slot = (unsigned long long*)(base + L.off_slot);
    sv.nwg = L.nwg;
    sv.pair_counts(ident.data(), g.n_r);
    const bool bipartite = lattice_bipartite(g);
    int n_even = 0;
    const std::vector<int32_t> order = colour_order(g, site_group(g), bipartite, &n_even);
    int* order_dev = (int*)(base + L.off_order);
    SCD_HIP(hipMemcpyAsync(order_dev, order.data(), (size_t)g.n_r * sizeof(int32_t),
                           hipMemcpyHostToDevice, st),
            "copy site order");
    sv.all_sites = order_dev;
    if (bipartite) {
        sv.colour_sites[0] = order_dev;
        sv.colour_sites[1] = order_dev + n_even;
        sv.n_colour[0] = n_even;
        sv.n_colour[1] = g.n_r - n_even;
    }

    const int e = t_index, be = 2 * g.n_real - 1 - t_index;
    double worst_err = 0.0, worst_rho = 0.0;
    double2* finals[2] = {nullptr, nullptr};
    for (int pass = 0; pass < (grads ? 2 : 1); ++pass) {
        SweepArgs a;
        a.Lx = g.Lx;
        a.Ly = g.Ly;
        a.periodic = g.periodic;
        a.n_r = g.n_r;
        a.n_t = g.n_t;
        a.ldx = L.ldx;
        a.ntn = L.ntn;
        a.bs = g.n_r;
        a.lc_sweep = 0;
        a.group = site_group(g);
        a.x0_kind = pass == 0 ? X0_COL : X0_COL_T;
        a.x0_fixed = pass == 0 ? be : e;
        a.sites = nullptr;
        a.n_sites = g.n_r;
        a.part_off = 0;
        a.check = 1;
        sv.St = pass == 0 ? St : StT;
        sv.St32 = prec != SCD_PREC_FP64 ? (void*)(base + (pass == 0 ? L.off_st32 : L.off_stt32))
                                        : nullptr;
        sv.bf3 = prec == SCD_PREC_BF16X3;
        double2* X = (double2*)(base + (pass == 0 ? L.off_xg : L.off_xh));
        double2* Xn = L.off_x1 ? (double2*)(base + L.off_x1) : nullptr;
        SCD_HIP(launch_init_block(g, (const double2*)S, src_dev, g.n_r, L.ldx, a.x0_kind,
                                  a.x0_fixed, X, Xn, st),
                "init launch");
        BlockResult res;
        int code;
        if (prec == SCD_PREC_FP64) {
            code = sv.solve_fp64(a, src_dev, X, Xn, tol, max_iter, &res);
        } else {
            code = sv.solve_mixed(a, src_dev, X, base + L.off_r32, base + L.off_d0,
                                  L.off_d1 ? base + L.off_d1 : nullptr, tol, max_iter, &res);
        }
        if (code == SCD_ENOTCONV)
            fail(SCD_ENOTCONV, "%s solve not converged after %d sweeps (e=%g)",
                 pass == 0 ? "forward" : "transposed", max_iter, res.err);
        stats.n_blocks++;
        stats.sweeps_total += res.sweeps;
        if (res.sweeps > stats.sweeps_max) stats.sweeps_max = res.sweeps;
        worst_err = std::max(worst_err, res.err);
        worst_rho = std::max(worst_rho, res.rho);
        if (code != SCD_OK) return finish(code);
        // The FP64 path ping-pongs; keep the final iterate where the gradient
        // kernels expect it.
        if (res.X != X)
            SCD_HIP(hipMemcpyAsync(X, res.X, (size_t)g.n_r * g.mp * L.ldx * sizeof(double2),
                                   hipMemcpyDeviceToDevice, st),
                    "iterate copy");
        finals[pass] = X;
    }
    SCD_HIP(launch_adjoint_loss(g, L.ldx, e, finals[0], w_loss, n_te, loss, st), "loss launch");
    if (grads) {
        SCD_HIP(launch_adjoint_grads(g, L.ldx, e, finals[1], finals[0], V, U, J, w_loss,
                                     (double2*)(base + L.off_lam), (double2*)(base + L.off_rsum),
                                     (double2*)(base + L.off_csum), (double*)(base + L.off_bz),
                                     (double*)(base + L.off_djc), dV, dU, dJ, st),
                "gradient launch");
    }
    SCD_HIP(hipStreamSynchronize(st), "final sync");
    stats.final_err = worst_err;
    stats.rho_est = worst_rho;
    g_last_error.clear();
    return finish(SCD_OK);
}

}  // extern "C"

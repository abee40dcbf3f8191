// Launch order of the sweep kernels' tiles (host side): which sites run
// together on an XCD, and in what order.  Kept apart from the rest of the host
// code because the order decides how much of the sweep kernel's traffic the
// caches absorb.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "internal.h"

namespace scd {

// Sites per tile-order group of the sweep kernel (see tile_site_col):
// SCD_SITE_GROUP overrides; the default keeps a group's site operands
// (mp^2 complex each) within about 2.7 MB of one XCD's 4 MB L2 (measured
// best on 16x16 / N_t = 144 and 24x24 / N_t = 176).
int site_group(const Geom& g) {
    if (const char* env = std::getenv("SCD_SITE_GROUP")) {
        const int v = std::atoi(env);
        if (v >= 1) return v < g.n_r ? v : g.n_r;
    }
    const double per_site = (double)g.mp * g.mp * 16.0;
    int grp = (int)(2.7e6 / per_site);
    if (grp < 1) grp = 1;
    if (grp > g.n_r) grp = g.n_r;
    return grp;
}

// Sites of the two colours of a bipartite lattice: (x + y) even, then odd.
// Within a colour, sites are listed patch by patch (square patches of
// `patch` x `patch` lattice sites, x-major inside), so that consecutive
// workgroups of one launch share the neighbour tiles of the other colour.
// SCD_PATCH overrides the default of 2 (a group of sites then covers a
// two-row strip of the lattice, whose targets share most neighbours).
int colour_patch(const Geom& g) {
    if (const char* env = std::getenv("SCD_PATCH")) {
        const int v = std::atoi(env);
        if (v >= 1) return v;
    }
    return 2;
}

// The sweep kernel hands each XCD one contiguous eighth of a launch's tile
// order, i.e. about one eighth of its site list.  Listing the site groups
// round-robin over the eight eighths (group k into eighth k mod 8) gives every
// XCD sites from all over the lattice, which keeps the XCDs balanced while the
// light cone (Sec. IV.D) still leaves the lattice's edges idle.  Whole groups
// move, so the sites that share an XCD's L2 stay neighbours; a partial group
// stays last.
static void interleave_groups(int32_t* sites, int n, int group) {
    const int full = n / group;
    std::vector<int32_t> out;
    out.reserve(n);
    for (int x = 0; x < 8; ++x)
        for (int k = x; k < full; k += 8)
            out.insert(out.end(), sites + (size_t)k * group, sites + (size_t)(k + 1) * group);
    out.insert(out.end(), sites + (size_t)full * group, sites + n);
    std::memcpy(sites, out.data(), (size_t)n * sizeof(int32_t));
}

// Launch site order.  Bipartite lattices: the two colours, (x + y) even then
// odd, each listed patch by patch (square patches of `patch` x `patch` sites,
// x-major inside) so that consecutive workgroups share the neighbour tiles of
// the other colour; *n_even is the size of the first colour.  Other lattices:
// all sites in index order, *n_even = 0.  Each segment is then interleaved
// over the XCDs in groups of `group` sites.
std::vector<int32_t> colour_order(const Geom& g, int group, bool bipartite, int* n_even) {
    const int patch = colour_patch(g);
    std::vector<int32_t> order;
    order.reserve(g.n_r);
    if (!bipartite) {
        for (int i = 0; i < g.n_r; ++i) order.push_back(i);
        *n_even = 0;
        interleave_groups(order.data(), g.n_r, group);
        return order;
    }
    for (int c = 0; c < 2; ++c) {
        for (int bx = 0; bx < g.Lx; bx += patch)
            for (int by = 0; by < g.Ly; by += patch)
                for (int x = bx; x < std::min(bx + patch, g.Lx); ++x)
                    for (int y = by; y < std::min(by + patch, g.Ly); ++y)
                        if ((x + y) % 2 == c) order.push_back(x * g.Ly + y);
        if (c == 0) *n_even = (int)order.size();
    }
    interleave_groups(order.data(), *n_even, group);
    interleave_groups(order.data() + *n_even, g.n_r - *n_even, group);
    return order;
}

}  // namespace scd

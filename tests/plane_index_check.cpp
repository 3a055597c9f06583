// Host enumeration of every index the elastic plane pass (plane_xy.hip) forms, with the
// same index functions (plane_index.h) the kernel uses: global loads of each tile's
// window, LDS window and result-tile indices, the nodes the patch solve asks the window
// for (chunk nodes, neighbour nodes and PMBC taps of both junctions, as x_unit reads
// them), and the epilogue's field offsets.  Usage:
//   plane_index_check nx ny nz Mx My halo periodic shots
// Prints "ok" and exits 0, or prints the first index out of its buffer and exits 1.
#include <cstdio>
#include <cstdlib>

#include "plane_index.h"

using namespace loss;

static int fails = 0;

static void check(bool ok, const char *what, long v, long lo, long hi)
{
    if (!ok && fails++ == 0) std::printf("%s = %ld outside [%ld, %ld)\n", what, v, lo, hi);
}

// the node a PMBC tap t of junction J reads (tap_node of the line kernels)
static int tap_node(int J, int t, int halo, int N, int periodic)
{
    int k = J - halo + t;
    if (periodic) k = k < 0 ? k + N : (k >= N ? k - N : k);
    else k = k < 0 ? 0 : (k > N ? N : k);
    return k;
}

// every node x_unit asks for when it solves patch sp of a line (G lanes, C nodes each)
template <typename F>
static void solve_requests(const Span &sp, int N, int halo, int periodic, int G, int C, F f)
{
    for (int k = 0; k < G; ++k) {
        const int q = sp.s + k * C;
        for (int c = 1; c <= C; ++c) f(q - 1 + c < N ? q - 1 + c : N);
        f(q + C < N ? q + C : N);
    }
    for (int t = 0; t < 2 * halo + 1; ++t) {
        f(tap_node(sp.s, t, halo, N, periodic));
        f(tap_node(sp.e, t, halo, N, periodic));
    }
}

int main(int argc, char **argv)
{
    if (argc != 9) {
        std::printf("usage: %s nx ny nz Mx My halo periodic shots\n", argv[0]);
        return 2;
    }
    const int N[3] = {atoi(argv[1]), atoi(argv[2]), atoi(argv[3])};
    const int Mx = atoi(argv[4]), My = atoi(argv[5]), halo = atoi(argv[6]), per = atoi(argv[7]);
    const int S = atoi(argv[8]);
    const int nx = N[0] + 1, ny = N[1] + 1, nz = N[2] + 1;
    const long pitch = (nx + 3) / 4 * 4, plane = pitch * ny, shot_stride = plane * nz;
    const long field = shot_stride * S;
    const int px = (N[0] + Mx - 1) / Mx, py = (N[1] + My - 1) / My;
    const int tile_side = 64 + 1;
    int Gx = 1, Gy = 1;
    while (Gx * kPlaneC < Mx) Gx <<= 1;
    while (Gy * kPlaneC < My) Gy <<= 1;
    // the launch's LDS size: two result tiles, then the window
    const int wxa = per ? Mx + 1 + 2 * halo : (N[0] + 1 < Mx + 1 + 2 * halo ? N[0] + 1 : Mx + 1 + 2 * halo);
    const int wya = per ? My + 1 + 2 * halo : (N[1] + 1 < My + 1 + 2 * halo ? N[1] + 1 : My + 1 + 2 * halo);
    const long lds_floats = 2L * tile_side * tile_side + (long)wxa * wya;
    const int load_slots = ((64 + 1 + 2 * 12) * (64 + 1 + 2 * 12) + kPlaneThreads - 1) / kPlaneThreads;
    for (int shot = 0; shot < S; ++shot)
        for (int z = 0; z < nz; z += (nz > 8 ? nz / 7 : 1)) {
            const long fbase = shot * shot_stride + z * plane;
            for (int ly = 0; ly < py; ++ly)
                for (int lx = 0; lx < px; ++lx) {
                    const Span sx = span_of(N[0], Mx, lx), sy = span_of(N[1], My, ly);
                    int wx0, wx1, wy0, wy1;
                    window_of(sx, N[0], halo, per, wx0, wx1);
                    window_of(sy, N[1], halo, per, wy0, wy1);
                    const int ww = wx1 - wx0 + 1, wh = wy1 - wy0 + 1;
                    check(ww <= wxa && wh <= wya, "window side", ww > wxa ? ww : wh, 0, ww > wxa ? wxa : wya);
                    check(sx.n <= tile_side && sy.n <= tile_side, "owned side", sx.n, 0, tile_side);
                    const int n = ww * wh;
                    check(n <= load_slots * kPlaneThreads, "window nodes", n, 0, load_slots * kPlaneThreads);
                    const float rw = 1.f / (float)ww;
                    for (int q = 0; q < load_slots * kPlaneThreads; ++q) {
                        int r, c;
                        split_flat(q < n - 1 ? q : n - 1, ww, rw, r, c);
                        check(r >= 0 && r < wh && c >= 0 && c < ww, "window split", q, 0, n);
                        const long g = fbase + (long)window_node(r, wy0, N[1]) * pitch + window_node(c, wx0, N[0]);
                        check(g >= 0 && g < field, "window load", g, 0, field);
                        check(window_node(c, wx0, N[0]) < nx && window_node(r, wy0, N[1]) < ny, "window node", c, 0, nx);
                        if (q < n) check(2L * tile_side * tile_side + q < lds_floats, "window store", q, 0, lds_floats);
                    }
                    // x lines of the owned rows, y lines of the owned columns
                    for (int r = 0; r < sy.n; ++r)
                        solve_requests(sx, N[0], halo, per, Gx, kPlaneC, [&](int i) {
                            const long idx = (long)(sy.s + r - wy0) * ww + window_pos(i, wx0, ww, N[0]);
                            check(idx >= 0 && idx < n, "row read", idx, 0, n);
                            // nodes the solve uses (the patch and its taps) must be the window's own
                            const int j = i - wx0;
                            const bool wrapped = j < 0 || j >= ww;
                            if (!per) check(!wrapped || i > sx.e, "row node outside window", i, wx0, wx1 + 1);
                        });
                    for (int c = 0; c < sx.n; ++c)
                        solve_requests(sy, N[1], halo, per, Gy, kPlaneC, [&](int i) {
                            const long idx = (long)window_pos(i, wy0, wh, N[1]) * ww + (sx.s + c - wx0);
                            check(idx >= 0 && idx < n, "column read", idx, 0, n);
                            const int j = i - wy0;
                            if (!per) check(!(j < 0 || j >= wh) || i > sy.e, "column node outside window", i, wy0, wy1 + 1);
                        });
                    // result tiles and the epilogue
                    const int nown = sy.n * sx.n;
                    const float rsn = 1.f / (float)sx.n;
                    for (int q = 0; q < nown; ++q) {
                        int r, c;
                        split_flat(q, sx.n, rsn, r, c);
                        check(r >= 0 && r < sy.n && c >= 0 && c < sx.n, "owned split", q, 0, nown);
                        check(r * tile_side + c < tile_side * tile_side, "result tile", r * tile_side + c, 0,
                              tile_side * tile_side);
                        const long off = (long)(sy.s + r) * pitch + sx.s + c;
                        check(sy.s + r < ny && sx.s + c < nx, "owned node", sx.s + c, 0, nx);
                        check(fbase + off < field, "field offset", fbase + off, 0, field);
                    }
                }
        }
    std::printf(fails ? "%d index(es) out of range\n" : "ok\n", fails);
    return fails ? 1 : 0;
}

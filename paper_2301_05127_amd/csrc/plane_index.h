// Index arithmetic of the elastic plane pass (plane_xy.hip), usable from host code so
// that a CPU check can enumerate every index the kernel forms for a given geometry.
#pragma once

#if defined(__HIPCC__)
#define LOSS_HD __host__ __device__ inline
#else
#define LOSS_HD inline
#endif

namespace loss {

constexpr int kPlaneThreads = 512;
constexpr int kPlaneC = 4;       // nodes per lane of the line solves

// patch nodes s..e of patch l of an axis with N intervals and patch length M; n owned
// nodes (e - s, and also N for the last patch)
struct Span {
    int s, e, n;
};

LOSS_HD Span span_of(int N, int M, int l)
{
    Span r;
    r.s = l * M;
    r.e = r.s + M < N ? r.s + M : N;
    r.n = r.e - r.s + (r.e == N ? 1 : 0);
    return r;
}

// (row, column) of flat element f of a region w wide, for 0 <= f < 2^14 (the float
// quotient is exact far below the 0.5 / w margin it needs)
LOSS_HD void split_flat(int f, int w, float rw, int &r, int &c)
{
    r = (int)(((float)f + 0.5f) * rw);
    c = f - r * w;
}

// Window of a tile along one axis: the patch nodes and the PMBC taps of its two
// junctions, clipped to [0, N], or on a periodic axis continued across the ends.
LOSS_HD void window_of(const Span &sp, int N, int halo, int periodic, int &w0, int &w1)
{
    w0 = sp.s - halo;
    w1 = sp.e + halo;
    if (!periodic) {
        w0 = w0 < 0 ? 0 : w0;
        w1 = w1 > N ? N : w1;
    }
}

// grid node at window coordinate w (past an end only on a periodic axis, where node N
// is node 0)
LOSS_HD int window_node(int w, int w0, int N)
{
    const int i = w0 + w;
    return i < 0 ? i + N : (i > N ? i - N : i);
}

// position in a window of wn nodes of node i of a line (a chunk node, or a PMBC tap that
// arrives wrapped into [0, N) on a periodic axis); clamped into the window, since the
// lanes of a patch shorter than G * C also ask for nodes past its closing node, whose
// values never reach a result
LOSS_HD int window_pos(int i, int w0, int wn, int N)
{
    int j = i - w0;
    j = j < 0 ? j + N : (j >= wn ? j - N : j);
    return j < 0 ? 0 : (j >= wn ? wn - 1 : j);
}

}  // namespace loss

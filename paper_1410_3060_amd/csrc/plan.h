// Diamond tiling of the (y, t) plane (Sect. 4.2, Fig. "diamond tiling") as
// used by the blocked scheme.
//
// With radius R, diamond width dw (a multiple of 2R, dw >= 4R) and
// half-height H = dw / (2R), row r of diamonds starts at t0 = r*H and its
// diamonds cover levels t0 + j, j = 1 .. 2H-1.  Diamond i of row r is centred
// at y_c = i*dw + (r odd ? dw/2 : 0); at level j it covers
//     y in [y_c - R*m(j), y_c + R*m(j)),   m(j) = min(j, 2H - j),
// so the edges have slope R cells per time step (S = +-1/R in the paper's
// notation) and the widest level (j = H) spans dw cells.  Consecutive rows are
// offset by dw/2 in y and by H in t; the diamonds of one row are independent
// and each depends on the two diamonds of the previous row that share its
// lower edges.  Rows are clipped to 1 <= t <= nt and diamonds to 0 <= y < ny
// (half diamonds at the y boundaries), so rows r = -1 .. floor((nt-1)/H)
// are needed.
//
// For a column y owned by diamond (r, i) (|y - y_c| within dw/2), with
// k = floor((y - y_c)/R) for y >= y_c and floor((y_c - y - 1)/R) otherwise,
// the diamond covers exactly the levels j = k+1 .. 2H-1-k.
#pragma once

#include <stdint.h>

#include <vector>

namespace stn {

struct diamond_row {
    int64_t r;          // row index (may be -1)
    int64_t t0;         // r * H
    int n_diamonds;     // diamonds whose ownership interval meets [0, ny)
    int first_centre;   // y_c of the first of them
};

struct diamond_plan {
    int R = 1, dw = 4, H = 2;
    std::vector<diamond_row> rows;
};

inline diamond_plan make_plan(int R, int dw, int ny, int64_t nt) {
    diamond_plan p;
    p.R = R;
    p.dw = dw;
    p.H = dw / (2 * R);
    if (nt <= 0 || ny <= 0) return p;
    const int64_t rmax = (nt - 1) / p.H;
    for (int64_t r = -1; r <= rmax; ++r) {
        diamond_row row;
        row.r = r;
        row.t0 = r * p.H;
        const bool odd = (r % 2) != 0;
        row.first_centre = odd ? dw / 2 : 0;
        // ownership [y_c - dw/2, y_c + dw/2) must meet [0, ny)
        int n = 0;
        for (int64_t yc = row.first_centre; yc - dw / 2 < ny; yc += dw) ++n;
        row.n_diamonds = n;
        p.rows.push_back(row);
    }
    return p;
}

}  // namespace stn

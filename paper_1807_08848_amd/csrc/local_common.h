// Device helpers of the local-solve kernels (k_local.hip, k_factor.hip,
// k_sweep.hip): boundary numbering of a buffered patch, the line view, and
// the bilinear-element stencil from the gathered coefficients.
#pragma once

#include "device_common.h"

namespace msrs {

// ------------------------------------------------------------ small helpers
// Counter-clockwise boundary index of local physical node (i, j) of a cx x cy
// cell block (caller guarantees the node is on the boundary).
__device__ __forceinline__ int bidx_ccw(int i, int j, int cx, int cy) {
    if (j == 0 && i < cx) return i;
    if (i == cx && j < cy) return cx + j;
    if (j == cy && i > 0) return cx + cy + (cx - i);
    return 2 * cx + cy + (cy - j);
}

// Local physical node (i, j) of counter-clockwise boundary index t (the
// inverse of bidx_ccw).
__device__ __forceinline__ void phys_of_bidx(int t, int cx, int cy, int& i, int& j) {
    if (t < cx) { i = t; j = 0; }
    else if (t < cx + cy) { i = cx; j = t - cx; }
    else if (t < 2 * cx + cy) { i = cx - (t - cx - cy); j = cy; }
    else { i = 0; j = cy - (t - 2 * cx - cy); }
}

// physical local node of line coordinates (p, q)
__device__ __forceinline__ void line_to_phys(const PatchDesc& P, int p, int q, int& i, int& j) {
    if (P.trans) { i = q; j = p; } else { i = p; j = q; }
}

// Row of the node at line coordinates (p, q) among the nodes of K_m
// (row-major, (nH + 1)^2 rows: the rows of Y and Q), or -1 outside K_m.
__device__ __forceinline__ int k_row_of(const PatchDesc& P, int p, int q) {
    int i, j;
    line_to_phys(P, p, q, i, j);
    const int ii = i - (P.kx0 - P.x0), jj = j - (P.ky0 - P.y0);
    return (ii >= 0 && ii <= P.nH && jj >= 0 && jj <= P.nH) ? jj * (P.nH + 1) + ii : -1;
}

__device__ __forceinline__ double a_cell(const double* aL, int L, int cr, int cp) { return aL[cr * L + cp]; }

// Q1 stencil coefficient between node (p,q) and (p+dp, q+dq) of a buffered
// patch, from the four elements around (p,q): NE=(p,q) NW=(p-1,q)
// SW=(p-1,q-1) SE=(p,q-1) (cell column, cell row).
__device__ __forceinline__ double q1_coef(const double* aL, int L, int p, int q, int dp, int dq) {
    const double NE = a_cell(aL, L, q, p), NW = a_cell(aL, L, q, p - 1);
    const double SW = a_cell(aL, L, q - 1, p - 1), SE = a_cell(aL, L, q - 1, p);
    if (dp == 0 && dq == 0) return (2.0 / 3.0) * (NE + NW + SW + SE);
    if (dq == 0) return dp > 0 ? -(NE + SE) / 6.0 : -(NW + SW) / 6.0;
    if (dp == 0) return dq > 0 ? -(NE + NW) / 6.0 : -(SE + SW) / 6.0;
    if (dp > 0) return dq > 0 ? -NE / 3.0 : -SE / 3.0;
    return dq > 0 ? -NW / 3.0 : -SW / 3.0;
}

static inline double dx_of(const Ctx& c) { return 1.0 / c.N; }

}  // namespace msrs

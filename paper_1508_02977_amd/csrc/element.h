// P1 element algebra on the pixel mesh, device side.
//
// Paper, Section 2.2 (weak form, two triangles per pixel) and Section 1
// (functional (BW2), rho = 0): per element K the local operator is
//   Lambda_c |K| grad phi_i . grad phi_j               (regulariser)
// + int_K a_c a_d phi_i phi_j,  a = (f_x, f_y, -f)      (data term)
// and the right-hand side -int_K f_t a_c phi_i, with f = I0 and f_t = I1 - I0
// both interpolated P1 and (f_x, f_y) the constant gradient of f on K.
//
// Cell (x, y) holds T0 = [(x,y), (x+1,y), (x+1,y+1)] and
// T1 = [(x,y), (x+1,y+1), (x,y+1)] (local vertex order 0, 1, 2).  All element
// integrals are exact: for |K| = 1/2,
//   int phi_i phi_j             = (1 + [i==j]) / 24
//   int phi_i phi_j phi_k       = 1/20, 1/60, 1/120   (3 equal, 2 equal, distinct)
//   int phi_i phi_j phi_k phi_l = 1/30, 1/120, 1/180, 1/360
//                                 (index multiplicities 4; 3+1; 2+2; 2+1+1).
#pragma once
#include <hip/hip_runtime.h>

namespace sfdd {

__host__ __device__ constexpr double mom2(int i, int j) { return i == j ? 1.0 / 12.0 : 1.0 / 24.0; }

__host__ __device__ constexpr double mom3(int i, int j, int k) {
    return (i == j && j == k) ? 1.0 / 20.0
         : (i == j || j == k || i == k) ? 1.0 / 60.0 : 1.0 / 120.0;
}

__host__ __device__ constexpr double mom4(int i, int j, int k, int l) {
    // multiplicities of vertex 0, 1, 2 among (i, j, k, l)
    int c0 = (i == 0) + (j == 0) + (k == 0) + (l == 0);
    int c1 = (i == 1) + (j == 1) + (k == 1) + (l == 1);
    int c2 = 4 - c0 - c1;
    int mx = c0 > c1 ? (c0 > c2 ? c0 : c2) : (c1 > c2 ? c1 : c2);
    int nz = (c0 > 0) + (c1 > 0) + (c2 > 0);
    return mx == 4 ? 1.0 / 30.0
         : mx == 3 ? 1.0 / 120.0
         : nz == 2 ? 1.0 / 180.0 : 1.0 / 360.0;
}

// |K| grad phi_i . grad phi_j for the unit right triangles T0 / T1.
__host__ __device__ constexpr double stiff(int t, int i, int j) {
    // T0: 1/2 [[1,-1,0],[-1,2,-1],[0,-1,1]];  T1: 1/2 [[1,0,-1],[0,1,-1],[-1,-1,2]]
    return t == 0 ? (i == j ? (i == 1 ? 1.0 : 0.5) : ((i + j == 1 || i + j == 3) ? -0.5 : 0.0))
                  : (i == j ? (i == 2 ? 1.0 : 0.5) : ((i == 2 || j == 2) ? -0.5 : 0.0));
}

// Node offsets (dx, dy) of the local vertices of T0 / T1 within cell (x, y).
__host__ __device__ constexpr int vdx(int t, int v) { return t == 0 ? (v == 0 ? 0 : 1) : (v == 1 ? 1 : 0); }
__host__ __device__ constexpr int vdy(int t, int v) { return t == 0 ? (v == 2 ? 1 : 0) : (v == 0 ? 0 : 1); }

// Image data of one element.
struct Elem {
    double f[3];   // P1 values of f = I0 at the vertices
    double gx, gy; // constant gradient of f on K
    double al;     // alpha_K
};

// f_x, f_y of the P1 interpolant on T0/T1 from the vertex values.
__device__ __forceinline__ void elem_grad(int t, const double f[3], double& gx, double& gy) {
    if (t == 0) { gx = f[1] - f[0]; gy = f[2] - f[1]; }
    else        { gx = f[1] - f[2]; gy = f[2] - f[0]; }
}

__device__ __forceinline__ Elem load_elem(const double* __restrict__ f0, const double* __restrict__ al,
                                          int W, int H, int cx, int cy, int t) {
    Elem e;
#pragma unroll
    for (int v = 0; v < 3; ++v) e.f[v] = f0[(cy + vdy(t, v)) * W + cx + vdx(t, v)];
    elem_grad(t, e.f, e.gx, e.gy);
    e.al = al[((size_t)cy * (W - 1) + cx) * 2 + t];
    return e;
}

// int f phi_i phi_j  (TT) and int f^2 phi_i phi_j (MM) for one row i.
__device__ __forceinline__ void elem_tt_row(const Elem& e, int i, double tt[3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s = fma(mom3(i, j, k), e.f[k], s);
        tt[j] = s;
    }
}

__device__ __forceinline__ void elem_mm_row(const Elem& e, int i, double mm[3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double sk = 0.0;
#pragma unroll
            for (int l = 0; l < 3; ++l) sk = fma(mom4(i, j, k, l), e.f[l], sk);
            s = fma(e.f[k], sk, s);
        }
        mm[j] = s;
    }
}

// Row (i, .) of the element operator applied to the element's vertex values
// u[v][c]:  out[c] = sum_{j,d} A_K[(i,c),(j,d)] u[j][d].
__device__ __forceinline__ void elem_apply_row(const Elem& e, int t, int i, const double u[3][3],
                                               double lam, double out[3]) {
    double tt[3], mm[3];
    elem_tt_row(e, i, tt);
    elem_mm_row(e, i, mm);
    double mgu = 0.0, ttm = 0.0, ttgu = 0.0, mmm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double gu = fma(e.gx, u[j][0], e.gy * u[j][1]);
        mgu = fma(mom2(i, j), gu, mgu);
        ttm = fma(tt[j], u[j][2], ttm);
        ttgu = fma(tt[j], gu, ttgu);
        mmm = fma(mm[j], u[j][2], mmm);
        double sij = stiff(t, i, j);
        s0 = fma(sij, u[j][0], s0);
        s1 = fma(sij, u[j][1], s1);
        s2 = fma(sij, u[j][2], s2);
    }
    double d = mgu - ttm;
    out[0] = fma(e.gx, d, e.al * s0);
    out[1] = fma(e.gy, d, e.al * s1);
    out[2] = mmm - ttgu + lam * s2;
}

// 3x3 block A_K[(i,.),(j,.)] (row field c, column field d), row-major.
__device__ __forceinline__ void elem_block(const Elem& e, int t, int i, int j, double lam, double blk[9]) {
    double tt[3], mm[3];
    elem_tt_row(e, i, tt);
    elem_mm_row(e, i, mm);
    const double g[2] = {e.gx, e.gy};
    const double mij = mom2(i, j), sij = stiff(t, i, j);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int d = 0; d < 2; ++d) blk[3 * c + d] = g[c] * g[d] * mij + (c == d ? e.al * sij : 0.0);
        blk[3 * c + 2] = -g[c] * tt[j];
        blk[6 + c] = -g[c] * tt[j];
    }
    blk[8] = mm[j] + lam * sij;
}

// Right-hand side of vertex i: out[c] = -int f_t a_c phi_i.
__device__ __forceinline__ void elem_rhs_row(const Elem& e, int i, const double ft[3], double out[3]) {
    double mft = 0.0, tft = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        mft = fma(mom2(i, k), ft[k], mft);
        double sk = 0.0;
#pragma unroll
        for (int l = 0; l < 3; ++l) sk = fma(mom3(i, k, l), ft[l], sk);
        tft = fma(e.f[k], sk, tft);
    }
    out[0] = -e.gx * mft;
    out[1] = -e.gy * mft;
    out[2] = tft;
}

// ---- smoothed data term (K_rho, Section 1) -------------------------------
//
// With the data term K_rho * (a a^T) and right-hand side -K_rho * (a f_t),
// K_rho a sampled normalised Gaussian over whole-pixel shifts s of the data
// (clamp to edge per axis), the element integrals are those above with every
// product of element data replaced by its weighted sum over the shifted
// elements K - s of the same type.  Per element 30 such sums (coefficient
// planes q):
//   q 0..2    G   = sum w g_c g_d            (xx, xy, yy)
//   q 3..8    GF  = sum w g_c f_k            (c = x: k = 0..2, then c = y)
//   q 9..14   FF  = sum w f_k f_l            (00, 01, 02, 11, 12, 22)
//   q 15..20  GT  = sum w g_c ft_k           (c = x: k = 0..2, then c = y)
//   q 21..29  FT  = sum w f_k ft_l           (k-major)
// (f_k, ft_k: vertex values of the shifted element in its local order).
constexpr int CLG_NCOEF = 30;

struct ElemC {
    double G[3], GF[2][3], FF[3][3], GT[2][3], FT[3][3];
    double al;
};

// The 30 products of one element's own data (before the shift sums).
__device__ __forceinline__ void clg_products(const double f[3], double gx, double gy, const double ft[3],
                                             double q[CLG_NCOEF]) {
    q[0] = gx * gx;
    q[1] = gx * gy;
    q[2] = gy * gy;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        q[3 + k] = gx * f[k];
        q[6 + k] = gy * f[k];
        q[15 + k] = gx * ft[k];
        q[18 + k] = gy * ft[k];
    }
    q[9] = f[0] * f[0];
    q[10] = f[0] * f[1];
    q[11] = f[0] * f[2];
    q[12] = f[1] * f[1];
    q[13] = f[1] * f[2];
    q[14] = f[2] * f[2];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) q[21 + 3 * k + l] = f[k] * ft[l];
}

// Coefficients of element e_id of a pair from planes [CLG_NCOEF][ne].
__device__ __forceinline__ ElemC load_elem_c(const double* __restrict__ coef, const double* __restrict__ al,
                                             int64_t ne, int64_t e_id) {
    ElemC c;
    auto q = [&](int i) { return coef[(int64_t)i * ne + e_id]; };
    c.G[0] = q(0);
    c.G[1] = q(1);
    c.G[2] = q(2);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c.GF[0][k] = q(3 + k);
        c.GF[1][k] = q(6 + k);
        c.GT[0][k] = q(15 + k);
        c.GT[1][k] = q(18 + k);
    }
    c.FF[0][0] = q(9);
    c.FF[0][1] = c.FF[1][0] = q(10);
    c.FF[0][2] = c.FF[2][0] = q(11);
    c.FF[1][1] = q(12);
    c.FF[1][2] = c.FF[2][1] = q(13);
    c.FF[2][2] = q(14);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) c.FT[k][l] = q(21 + 3 * k + l);
    c.al = al[e_id];
    return c;
}

// int (sum w g_c f) phi_i phi_j = sum_k mom3(i,j,k) GF_ck, and
// int (sum w f f) phi_i phi_j = sum_kl mom4(i,j,k,l) FF_kl, for one row i.
__device__ __forceinline__ void elemc_rows(const ElemC& e, int i, double tt[2][3], double mm[3]) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        double s0 = 0.0, s1 = 0.0, sm = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s0 = fma(mom3(i, j, k), e.GF[0][k], s0);
            s1 = fma(mom3(i, j, k), e.GF[1][k], s1);
#pragma unroll
            for (int l = 0; l < 3; ++l) sm = fma(mom4(i, j, k, l), e.FF[k][l], sm);
        }
        tt[0][j] = s0;
        tt[1][j] = s1;
        mm[j] = sm;
    }
}

// Row (i, .) of the smoothed element operator applied to u[v][c] (as elem_apply_row).
__device__ __forceinline__ void elemc_apply_row(const ElemC& e, int t, int i, const double u[3][3], double lam,
                                                double out[3]) {
    double tt[2][3], mm[3];
    elemc_rows(e, i, tt, mm);
    double o0 = 0.0, o1 = 0.0, o2 = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const double mij = mom2(i, j);
        o0 += mij * (e.G[0] * u[j][0] + e.G[1] * u[j][1]) - tt[0][j] * u[j][2];
        o1 += mij * (e.G[1] * u[j][0] + e.G[2] * u[j][1]) - tt[1][j] * u[j][2];
        o2 += mm[j] * u[j][2] - tt[0][j] * u[j][0] - tt[1][j] * u[j][1];
        const double sij = stiff(t, i, j);
        s0 = fma(sij, u[j][0], s0);
        s1 = fma(sij, u[j][1], s1);
        s2 = fma(sij, u[j][2], s2);
    }
    out[0] = fma(e.al, s0, o0);
    out[1] = fma(e.al, s1, o1);
    out[2] = fma(lam, s2, o2);
}

// 3x3 block of the smoothed element operator (as elem_block).
__device__ __forceinline__ void elemc_block(const ElemC& e, int t, int i, int j, double lam, double blk[9]) {
    double tt[2][3], mm[3];
    elemc_rows(e, i, tt, mm);
    const double mij = mom2(i, j), sij = stiff(t, i, j);
    const double G[2][2] = {{e.G[0], e.G[1]}, {e.G[1], e.G[2]}};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int d = 0; d < 2; ++d) blk[3 * c + d] = G[c][d] * mij + (c == d ? e.al * sij : 0.0);
        blk[3 * c + 2] = -tt[c][j];
        blk[6 + c] = -tt[c][j];
    }
    blk[8] = mm[j] + lam * sij;
}

// Right-hand side of vertex i with the smoothed data (as elem_rhs_row).
__device__ __forceinline__ void elemc_rhs_row(const ElemC& e, int i, double out[3]) {
    double r0 = 0.0, r1 = 0.0, r2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r0 = fma(mom2(i, k), e.GT[0][k], r0);
        r1 = fma(mom2(i, k), e.GT[1][k], r1);
#pragma unroll
        for (int l = 0; l < 3; ++l) r2 = fma(mom3(i, k, l), e.FT[k][l], r2);
    }
    out[0] = -r0;
    out[1] = -r1;
    out[2] = r2;
}

// The six elements around node (x, y): cell offset and local vertex index.
//   T0 of cells (x,y) [v0], (x-1,y) [v1], (x-1,y-1) [v2]
//   T1 of cells (x,y) [v0], (x-1,y-1) [v1], (x,y-1) [v2]
struct Around { int dcx, dcy, t, v; };
__host__ __device__ constexpr Around around(int k) {
    return k == 0 ? Around{0, 0, 0, 0}
         : k == 1 ? Around{-1, 0, 0, 1}
         : k == 2 ? Around{-1, -1, 0, 2}
         : k == 3 ? Around{0, 0, 1, 0}
         : k == 4 ? Around{-1, -1, 1, 1}
                  : Around{0, -1, 1, 2};
}

// 3x3 block A[(x,y), (x+dx, y+dy)] of the global matrix, row field c,
// column field d, for (dx, dy) in {(0,0), (1,0), (0,1), (1,1)}.  With
// coef != nullptr the data term is the smoothed one of the coefficient
// planes coef [CLG_NCOEF][(W-1)(H-1)2] of this pair.
__device__ inline void stencil_block(const double* __restrict__ f0, const double* __restrict__ al, int W, int H,
                              int x, int y, int dx, int dy, double lam, double blk[9],
                              const double* __restrict__ coef = nullptr) {
    for (int i = 0; i < 9; ++i) blk[i] = 0.0;
    double b[9];
    const int64_t ne = (int64_t)(W - 1) * (H - 1) * 2;
    auto add = [&](int cx, int cy, int t, int i, int j) {
        if (cx < 0 || cy < 0 || cx >= W - 1 || cy >= H - 1) return;
        if (coef) {
            const ElemC e = load_elem_c(coef, al, ne, ((int64_t)cy * (W - 1) + cx) * 2 + t);
            elemc_block(e, t, i, j, lam, b);
        } else {
            Elem e = load_elem(f0, al, W, H, cx, cy, t);
            elem_block(e, t, i, j, lam, b);
        }
        for (int k = 0; k < 9; ++k) blk[k] += b[k];
    };
    if (dx == 0 && dy == 0) {
        for (int k = 0; k < 6; ++k) {
            const Around a = around(k);
            add(x + a.dcx, y + a.dcy, a.t, a.v, a.v);
        }
    } else if (dx == 1 && dy == 0) {          // edge (x,y)-(x+1,y)
        add(x, y, 0, 0, 1);
        add(x, y - 1, 1, 2, 1);
    } else if (dx == 0 && dy == 1) {          // edge (x,y)-(x,y+1)
        add(x, y, 1, 0, 2);
        add(x - 1, y, 0, 1, 2);
    } else {                                  // diagonal edge (x,y)-(x+1,y+1)
        add(x, y, 0, 0, 2);
        add(x, y, 1, 0, 1);
    }
}

}  // namespace sfdd

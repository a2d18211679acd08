// Matrix-free P1 kernels: input validation, right-hand side, residual,
// residual error indicator and the alpha update.  One thread per node (or
// per element); every reduction is a fixed-order two-stage sum, so results
// are bitwise reproducible run to run.
#include <cmath>
#include <mutex>

#include "element.h"
#include "sfdd_internal.h"

namespace sfdd {

constexpr int NODE_THREADS = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    // fixed-order reduction over the block (deterministic)
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
    return s;
}

__global__ void k_validate(const double* __restrict__ I0, const double* __restrict__ I1,
                           const double* __restrict__ al, int64_t nn, int64_t ne, int32_t* flags) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int bad_img = 0, bad_al = 0;
    for (int64_t k = i; k < nn; k += stride)
        if (!isfinite(I0[k]) || !isfinite(I1[k])) bad_img = 1;
    for (int64_t k = i; k < ne; k += stride)
        if (!isfinite(al[k]) || !(al[k] > 0.0)) bad_al = 1;
    if (bad_img) atomicOr(&flags[0], 1);
    if (bad_al) atomicOr(&flags[1], 1);
}

// Copies f0 = I0, ft = I1 - I0, alpha; F = -int f_t a phi_i; ||F||^2 partials.
__global__ void k_assemble(const double* __restrict__ I0, const double* __restrict__ I1,
                           const double* __restrict__ al_in, double* __restrict__ f0,
                           double* __restrict__ ft, double* __restrict__ al, double* __restrict__ F,
                           double* __restrict__ partials, int npart, int W, int H) {
    __shared__ double sh[NODE_THREADS / 64];
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const double* i0 = I0 + pair * nn;
    const double* i1 = I1 + pair * nn;
    const double* ali = al_in + pair * ne;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (node < nn) {
        f0[pair * nn + node] = i0[node];
        ft[pair * nn + node] = i1[node] - i0[node];
        for (int k = 0; k < 2; ++k) {
            int64_t e = 2 * (int64_t)node + k;
            if (e < ne) al[pair * ne + e] = ali[e];
        }
        const int x = node % W, y = node / W;
        double out[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const Around a = around(k);
            const int cx = x + a.dcx, cy = y + a.dcy;
            if (cx < 0 || cy < 0 || cx >= W - 1 || cy >= H - 1) continue;
            Elem e = load_elem(i0, ali, W, H, cx, cy, a.t);
            double ftv[3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const int n = (cy + vdy(a.t, v)) * W + cx + vdx(a.t, v);
                ftv[v] = i1[n] - i0[n];
            }
            double o[3];
            elem_rhs_row(e, a.v, ftv, o);
            out[0] += o[0];
            out[1] += o[1];
            out[2] += o[2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) F[(pair * 3 + c) * nn + node] = out[c];
        acc = out[0] * out[0] + out[1] * out[1] + out[2] * out[2];
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[pair * npart + blockIdx.x] = s;
}

__global__ void k_finalize_norm(const double* __restrict__ partials, int npart, double* __restrict__ out) {
    const int pair = blockIdx.x;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < npart; ++i) s += partials[pair * npart + i];
        out[pair] = s;
    }
}

// r = F - A U and ||r||^2 partials; pairs already converged are skipped.
template <bool CLG>
__global__ void k_residual(const double* __restrict__ f0, const double* __restrict__ al,
                           const double* __restrict__ F, const double* __restrict__ U,
                           double* __restrict__ r, double* __restrict__ partials, int npart,
                           int W, int H, double lam, const int32_t* __restrict__ done,
                           const double* __restrict__ coef) {
    __shared__ double sh[NODE_THREADS / 64];
    const int pair = blockIdx.y;
    if (done != nullptr && done[pair]) {
        if (threadIdx.x == 0) partials[pair * npart + blockIdx.x] = 0.0;
        return;
    }
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const double* fp = f0 + pair * nn;
    const double* ap = al + pair * ne;
    const double* Up = U + pair * 3 * nn;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (node < nn) {
        const int x = node % W, y = node / W;
        double out[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] = F[(pair * 3 + c) * nn + node];
        // plain data term: branch-free over the six elements (so that all
        // their loads are in flight together): an element outside the image
        // is evaluated on the nearest cell and contributes an exact zero
        // (x - 0 = x, so the sum is the one over the elements that exist, in
        // the same order).  The smoothed term (more loads per element) keeps
        // the skip, which needs fewer registers.
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const Around a = around(k);
            const int cx0 = x + a.dcx, cy0 = y + a.dcy;
            const bool inside = cx0 >= 0 && cy0 >= 0 && cx0 < W - 1 && cy0 < H - 1;
            if (CLG && !inside) continue;
            const int cx = min(max(cx0, 0), W - 2), cy = min(max(cy0, 0), H - 2);
            double u[3][3];
#pragma unroll
            for (int v = 0; v < 3; ++v) {
                const int64_t n = (int64_t)(cy + vdy(a.t, v)) * W + cx + vdx(a.t, v);
#pragma unroll
                for (int c = 0; c < 3; ++c) u[v][c] = Up[c * nn + n];
            }
            double o[3];
            if constexpr (CLG) {
                const ElemC e = load_elem_c(coef + (int64_t)pair * CLG_NCOEF * ne, ap, ne,
                                            ((int64_t)cy * (W - 1) + cx) * 2 + a.t);
                elemc_apply_row(e, a.t, a.v, u, lam, o);
            } else {
                Elem e = load_elem(fp, ap, W, H, cx, cy, a.t);
                elem_apply_row(e, a.t, a.v, u, lam, o);
            }
            out[0] -= inside ? o[0] : 0.0;
            out[1] -= inside ? o[1] : 0.0;
            out[2] -= inside ? o[2] : 0.0;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) r[(pair * 3 + c) * nn + node] = out[c];
        acc = out[0] * out[0] + out[1] * out[1] + out[2] * out[2];
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[pair * npart + blockIdx.x] = s;
}

// Stop test of sweep `sweep` (checked before the sweep): per pair relres =
// ||r||/||F||; a pair stops when relres <= rtol, on F = 0, on a non-finite
// norm or when sweep == max_sweeps.  Also clears the sweep counters.
// Stop test, one block per pair: ||r||^2 from the residual kernel's block
// partials (fixed-order reduction), relres = ||r|| / ||F||; a pair stops at
// relres <= rtol, on a non-finite norm, at max_sweeps, or at once if F = 0.
__global__ void k_converge(const double* __restrict__ partials, int npart, const double* __restrict__ Fn2,
                           double* __restrict__ relres, int32_t* __restrict__ sweeps,
                           int32_t* __restrict__ done, double rtol, int sweep, int max_sweeps,
                           const int32_t* __restrict__ sweep_dev) {
    __shared__ double sh[NODE_THREADS / 64];
    const int pair = blockIdx.x;
    if (done[pair]) return;                      // uniform over the block
    if (sweep_dev) sweep = *sweep_dev;           // graph replay: the index lives on the device
    double v = 0.0;
    for (int i = threadIdx.x; i < npart; i += blockDim.x) v += partials[(int64_t)pair * npart + i];
    const double s = block_sum(v, sh);
    if (threadIdx.x == 0) {
        const double fn = Fn2[pair];
        double rel;
        int stop;
        if (fn == 0.0) { rel = 0.0; stop = 1; }
        else {
            rel = sqrt(s) / sqrt(fn);
            stop = !isfinite(rel) || rel <= rtol || sweep >= max_sweeps;
        }
        relres[pair] = rel;
        sweeps[pair] = sweep;
        if (stop) done[pair] = 1;
    }
}

// --- smoothed data term K_rho (Section 1) ---------------------------------
//
// The 30 coefficient planes of every element (element.h): the weighted sums
// over whole-pixel shifts s of the products of the shifted element's data,
// K - s of the same type, the cell index clamped to the cell grid per axis.
// The weights are separable, so the sums run in two passes: along x (the
// products formed on the fly from f0 and ft) into tmp, then along y into coef.
// Both arrays are [B][CLG_NCOEF][ne].

__device__ __forceinline__ void elem_products(const double* __restrict__ fp, const double* __restrict__ tp, int W,
                                              int cx, int cy, int t, double q[CLG_NCOEF]) {
    double f[3], ft[3], gx, gy;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const int64_t n = (int64_t)(cy + vdy(t, v)) * W + cx + vdx(t, v);
        f[v] = fp[n];
        ft[v] = tp[n];
    }
    elem_grad(t, f, gx, gy);
    clg_products(f, gx, gy, ft, q);
}

__global__ void k_clg_smooth_x(const double* __restrict__ f0, const double* __restrict__ ft,
                               const double* __restrict__ w, int r, double* __restrict__ tmp, int W, int H) {
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const int64_t e_id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e_id >= ne) return;
    const int t = (int)(e_id & 1), cell = (int)(e_id >> 1);
    const int cx = cell % (W - 1), cy = cell / (W - 1);
    double acc[CLG_NCOEF];
#pragma unroll
    for (int q = 0; q < CLG_NCOEF; ++q) acc[q] = 0.0;
    for (int k = -r; k <= r; ++k) {
        const int sx = min(max(cx - k, 0), W - 2);
        double q[CLG_NCOEF];
        elem_products(f0 + pair * nn, ft + pair * nn, W, sx, cy, t, q);
        const double wk = w[k + r];
#pragma unroll
        for (int i = 0; i < CLG_NCOEF; ++i) acc[i] = fma(wk, q[i], acc[i]);
    }
    double* out = tmp + (int64_t)pair * CLG_NCOEF * ne + e_id;
#pragma unroll
    for (int q = 0; q < CLG_NCOEF; ++q) out[(int64_t)q * ne] = acc[q];
}

__global__ void k_clg_smooth_y(const double* __restrict__ tmp, const double* __restrict__ w, int r,
                               double* __restrict__ coef, int W, int H) {
    const int pair = blockIdx.z, q = blockIdx.y;
    const int64_t ne = (int64_t)(W - 1) * (H - 1) * 2;
    const int64_t e_id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e_id >= ne) return;
    const int64_t row = 2 * (int64_t)(W - 1);            // elements per cell row
    const int cy = (int)(e_id / row);
    const double* in = tmp + ((int64_t)pair * CLG_NCOEF + q) * ne + (e_id - cy * row);
    double acc = 0.0;
    for (int k = -r; k <= r; ++k) {
        const int sy = min(max(cy - k, 0), H - 2);
        acc = fma(w[k + r], in[sy * row], acc);
    }
    coef[((int64_t)pair * CLG_NCOEF + q) * ne + e_id] = acc;
}

// F with the smoothed data (replaces k_assemble's F) and ||F||^2 partials.
__global__ void k_clg_rhs(const double* __restrict__ coef, const double* __restrict__ al, double* __restrict__ F,
                          double* __restrict__ partials, int npart, int W, int H) {
    __shared__ double sh[NODE_THREADS / 64];
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const int node = blockIdx.x * blockDim.x + threadIdx.x;
    double acc = 0.0;
    if (node < nn) {
        const int x = node % W, y = node / W;
        double out[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const Around a = around(k);
            const int cx = x + a.dcx, cy = y + a.dcy;
            if (cx < 0 || cy < 0 || cx >= W - 1 || cy >= H - 1) continue;
            const ElemC e = load_elem_c(coef + (int64_t)pair * CLG_NCOEF * ne, al + pair * ne, ne,
                                        ((int64_t)cy * (W - 1) + cx) * 2 + a.t);
            double o[3];
            elemc_rhs_row(e, a.v, o);
            out[0] += o[0];
            out[1] += o[1];
            out[2] += o[2];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) F[(pair * 3 + c) * nn + node] = out[c];
        acc = out[0] * out[0] + out[1] * out[1] + out[2] * out[2];
    }
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[pair * npart + blockIdx.x] = s;
}

// --- residual error indicator (Section 2.3) -------------------------------
//
// eta_K = alpha_K^{-1/2} h_K |grad f| (int_K (s + f_t)^2)^{1/2}
//       + 1/2 sum_e alpha_e^{-1/2} h_e |[alpha grad u . n_e]|,
// s = f_x u1 + f_y u2 - f m, flow components only, alpha_e = max over the two
// elements of e (own alpha on the image border, outside flux 0).
// The degree-4 element integral uses the 6-point rule with points
// (a, a, 1-2a) for a = a1, a2 and weights w1, w2 (sum of weights 1, exact to
// degree 4, all weights positive), so the integral is a sum of squares.

__device__ __forceinline__ void flux_grad(int t, const double u[3], double& dx, double& dy) {
    if (t == 0) { dx = u[1] - u[0]; dy = u[2] - u[1]; }
    else        { dx = u[1] - u[2]; dy = u[2] - u[0]; }
}

__device__ void elem_flux(const double* __restrict__ Up, int64_t nn, int W, int cx, int cy, int t,
                          double al, double flux[2][2]) {
    for (int c = 0; c < 2; ++c) {
        double u[3];
        for (int v = 0; v < 3; ++v) u[v] = Up[c * nn + (int64_t)(cy + vdy(t, v)) * W + cx + vdx(t, v)];
        double gx, gy;
        flux_grad(t, u, gx, gy);
        flux[c][0] = al * gx;
        flux[c][1] = al * gy;
    }
}

__global__ void k_indicator(const double* __restrict__ f0, const double* __restrict__ ft,
                            const double* __restrict__ al, const double* __restrict__ U,
                            double* __restrict__ eta, uint64_t* __restrict__ etamax_bits, int W, int H,
                            const double* __restrict__ coef) {
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const int64_t e_id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e_id >= ne) return;
    const int t = (int)(e_id & 1);
    const int cell = (int)(e_id >> 1);
    const int cx = cell % (W - 1), cy = cell / (W - 1);
    const double* fp = f0 + pair * nn;
    const double* tp = ft + pair * nn;
    const double* ap = al + pair * ne;
    const double* Up = U + pair * 3 * nn;
    Elem e = load_elem(fp, ap, W, H, cx, cy, t);
    double ftv[3], uv[3][3];
    for (int v = 0; v < 3; ++v) {
        const int64_t n = (int64_t)(cy + vdy(t, v)) * W + cx + vdx(t, v);
        ftv[v] = tp[n];
        for (int c = 0; c < 3; ++c) uv[v][c] = Up[c * nn + n];
    }
    // element residual: int_K (s + f_t)^2, |K| = 1/2
    const double qa[2] = {0.44594849091596489, 0.091576213509770743};
    const double qw[2] = {0.22338158967801147, 0.10995174365532187};
    double quad = 0.0;
    for (int g = 0; g < 2; ++g) {
        const double a = qa[g], b = 1.0 - 2.0 * a;
        for (int p = 0; p < 3; ++p) {
            double l[3] = {a, a, a};
            l[p] = b;
            double f = 0.0, ftq = 0.0, u1 = 0.0, u2 = 0.0, m = 0.0;
            for (int v = 0; v < 3; ++v) {
                f = fma(l[v], e.f[v], f);
                ftq = fma(l[v], ftv[v], ftq);
                u1 = fma(l[v], uv[v][0], u1);
                u2 = fma(l[v], uv[v][1], u2);
                m = fma(l[v], uv[v][2], m);
            }
            const double val = e.gx * u1 + e.gy * u2 - f * m + ftq;
            quad = fma(qw[g] * val, val, quad);
        }
    }
    quad *= 0.5;
    const double sq2 = 1.4142135623730951;
    double res = sq2 * sqrt((e.gx * e.gx + e.gy * e.gy) * quad) / sqrt(e.al);
    if (coef) {
        // smoothed data: R_c = sum_d G_cd u_d - m sum_k GF_ck phi_k + sum_k GT_ck phi_k
        // (c = x, y), int_K R_x^2 + R_y^2 by the same rule
        const ElemC ec = load_elem_c(coef + (int64_t)pair * CLG_NCOEF * ne, ap, ne, e_id);
        double qc = 0.0;
        for (int g = 0; g < 2; ++g) {
            const double a = qa[g], b = 1.0 - 2.0 * a;
            for (int p = 0; p < 3; ++p) {
                double l[3] = {a, a, a};
                l[p] = b;
                double u1 = 0.0, u2 = 0.0, m = 0.0, gf0 = 0.0, gf1 = 0.0, gt0 = 0.0, gt1 = 0.0;
                for (int v = 0; v < 3; ++v) {
                    u1 = fma(l[v], uv[v][0], u1);
                    u2 = fma(l[v], uv[v][1], u2);
                    m = fma(l[v], uv[v][2], m);
                    gf0 = fma(l[v], ec.GF[0][v], gf0);
                    gf1 = fma(l[v], ec.GF[1][v], gf1);
                    gt0 = fma(l[v], ec.GT[0][v], gt0);
                    gt1 = fma(l[v], ec.GT[1][v], gt1);
                }
                const double r0 = ec.G[0] * u1 + ec.G[1] * u2 - gf0 * m + gt0;
                const double r1 = ec.G[1] * u1 + ec.G[2] * u2 - gf1 * m + gt1;
                qc = fma(qw[g], r0 * r0 + r1 * r1, qc);
            }
        }
        res = sq2 * sqrt(0.5 * qc) / sqrt(e.al);
    }
    // flux jumps over the three edges
    double fin[2][2];
    elem_flux(Up, nn, W, cx, cy, t, e.al, fin);
    for (int k = 0; k < 3; ++k) {
        // neighbour cell / type and unit normal of edge k
        int ncx, ncy, nt;
        double nx, ny, he;
        if (t == 0) {
            if (k == 0)      { ncx = cx;     ncy = cy - 1; nt = 1; nx = 0.0;  ny = -1.0; he = 1.0; }  // bottom
            else if (k == 1) { ncx = cx + 1; ncy = cy;     nt = 1; nx = 1.0;  ny = 0.0;  he = 1.0; }  // right
            else             { ncx = cx;     ncy = cy;     nt = 1; nx = -0.70710678118654752; ny = 0.70710678118654752; he = sq2; }
        } else {
            if (k == 0)      { ncx = cx;     ncy = cy + 1; nt = 0; nx = 0.0;  ny = 1.0;  he = 1.0; }  // top
            else if (k == 1) { ncx = cx - 1; ncy = cy;     nt = 0; nx = -1.0; ny = 0.0;  he = 1.0; }  // left
            else             { ncx = cx;     ncy = cy;     nt = 0; nx = 0.70710678118654752; ny = -0.70710678118654752; he = sq2; }
        }
        double fout[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        double ae = e.al;
        if (ncx >= 0 && ncy >= 0 && ncx < W - 1 && ncy < H - 1) {
            const double an = ap[((int64_t)ncy * (W - 1) + ncx) * 2 + nt];
            elem_flux(Up, nn, W, ncx, ncy, nt, an, fout);
            ae = fmax(ae, an);
        }
        const double j0 = (fout[0][0] - fin[0][0]) * nx + (fout[0][1] - fin[0][1]) * ny;
        const double j1 = (fout[1][0] - fin[1][0]) * nx + (fout[1][1] - fin[1][1]) * ny;
        res += 0.5 * he * sqrt(j0 * j0 + j1 * j1) / sqrt(ae);
    }
    eta[pair * ne + e_id] = res;
    // eta >= 0, so the IEEE bit pattern orders like an unsigned integer
    atomicMax((unsigned long long*)&etamax_bits[pair], (unsigned long long)__double_as_longlong(res));
}

__global__ void k_alpha_update(const double* __restrict__ eta, const uint64_t* __restrict__ etamax_bits,
                               double* __restrict__ al, double* __restrict__ al_out, int64_t ne,
                               double kappa, double eta_thr, double alpha_th) {
    const int pair = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const double mx = __longlong_as_double((long long)etamax_bits[pair]);
    const double a = al[pair * ne + i];
    double an = a;
    if (mx > 0.0) {
        const double rel = eta[pair * ne + i] / mx;
        an = fmax(a / (1.0 + kappa * fmax(rel - eta_thr, 0.0)), alpha_th);
    }
    al[pair * ne + i] = an;
    al_out[pair * ne + i] = an;
}

__global__ void k_zero_u64(uint64_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ---- launchers -----------------------------------------------------------

#define SF_LAUNCH_CHECK()                                   \
    do {                                                    \
        if (hipGetLastError() != hipSuccess) return SF_ERR_HIP; \
    } while (0)

// --- adjoint gradients ------------------------------------------------------
// For a loss L(U) of the solution of A(theta) U = F(theta) and the adjoint
// state P (A P = dL/dU, A symmetric), dL/dtheta = -d/dtheta [P^T (A U - F)] at
// fixed U, P.  P^T (A U - F) = sum_K int_K (a.P)(a.U + f_t) + alpha_K
// (grad P1.grad U1 + grad P2.grad U2) + lambda grad P3.grad U3, a = (f_x, f_y, -f).

// dL/dalpha_K = -|K| sum_{c=1,2} grad P_c . grad U_c, one thread per element
__global__ void k_adj_alpha(const double* __restrict__ U, const double* __restrict__ P, double* __restrict__ dal,
                            int W, int H) {
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const int64_t e_id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e_id >= ne) return;
    const int t = (int)(e_id & 1), cell = (int)(e_id >> 1);
    const int cx = cell % (W - 1), cy = cell / (W - 1);
    const double* Up = U + pair * 3 * nn;
    const double* Pp = P + pair * 3 * nn;
    int64_t nv[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) nv[v] = (int64_t)(cy + vdy(t, v)) * W + cx + vdx(t, v);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double su = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) su = fma(stiff(t, i, j), Up[c * nn + nv[j]], su);
            s = fma(Pp[c * nn + nv[i]], su, s);
        }
    dal[pair * ne + e_id] = -s;
}

// gradient of the P1 basis function of local vertex v on T0 / T1
__device__ __forceinline__ void basis_grad(int t, int v, double& gx, double& gy) {
    if (t == 0) { gx = v == 0 ? -1.0 : (v == 1 ? 1.0 : 0.0); gy = v == 1 ? -1.0 : (v == 2 ? 1.0 : 0.0); }
    else        { gx = v == 1 ? 1.0 : (v == 2 ? -1.0 : 0.0); gy = v == 0 ? -1.0 : (v == 2 ? 1.0 : 0.0); }
}

// dL/dI1_n = -sum_K int_K p phi_n and
// dL/dI0_n = -sum_K int_K (grad phi_n.(P1,P2) - phi_n P3) e + p (grad phi_n.(U1,U2) - phi_n U3 - phi_n)
// with p = a.P, e = a.U + f_t: a gather over the six elements around node n,
// each integrand (degree <= 4) by the 6-point degree-4 Dunavant rule.
__global__ void k_adj_frames(const double* __restrict__ f0, const double* __restrict__ ft,
                             const double* __restrict__ U, const double* __restrict__ P,
                             double* __restrict__ dI0, double* __restrict__ dI1, int W, int H) {
    const int pair = blockIdx.y;
    const int64_t nn = (int64_t)W * H;
    const int64_t node = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (node >= nn) return;
    const int x = (int)(node % W), y = (int)(node / W);
    const double* fp = f0 + pair * nn;
    const double* tp = ft + pair * nn;
    const double* Up = U + pair * 3 * nn;
    const double* Pp = P + pair * 3 * nn;
    const double qa[2] = {0.44594849091596489, 0.091576213509770743};
    const double qw[2] = {0.22338158967801147, 0.10995174365532187};
    double s0 = 0.0, s1 = 0.0;
    for (int k = 0; k < 6; ++k) {
        const Around a = around(k);
        const int cx = x + a.dcx, cy = y + a.dcy;
        if (cx < 0 || cy < 0 || cx >= W - 1 || cy >= H - 1) continue;
        double fv[3], tv[3], uv[3][3], pv[3][3];
        for (int v = 0; v < 3; ++v) {
            const int64_t n = (int64_t)(cy + vdy(a.t, v)) * W + cx + vdx(a.t, v);
            fv[v] = fp[n];
            tv[v] = tp[n];
            for (int c = 0; c < 3; ++c) {
                uv[v][c] = Up[c * nn + n];
                pv[v][c] = Pp[c * nn + n];
            }
        }
        double gx, gy, bx, by;
        elem_grad(a.t, fv, gx, gy);
        basis_grad(a.t, a.v, bx, by);
        for (int g = 0; g < 2; ++g) {
            const double qa_ = qa[g], qb = 1.0 - 2.0 * qa_;
            for (int q = 0; q < 3; ++q) {
                double l[3] = {qa_, qa_, qa_};
                l[q] = qb;
                double f = 0.0, ftq = 0.0, u[3] = {0.0, 0.0, 0.0}, pq[3] = {0.0, 0.0, 0.0};
                for (int v = 0; v < 3; ++v) {
                    f = fma(l[v], fv[v], f);
                    ftq = fma(l[v], tv[v], ftq);
                    for (int c = 0; c < 3; ++c) {
                        u[c] = fma(l[v], uv[v][c], u[c]);
                        pq[c] = fma(l[v], pv[v][c], pq[c]);
                    }
                }
                const double phi = l[a.v];
                const double p = gx * pq[0] + gy * pq[1] - f * pq[2];
                const double e = gx * u[0] + gy * u[1] - f * u[2] + ftq;
                const double w = 0.5 * qw[g];                         // |K| = 1/2
                s1 = fma(w, p * phi, s1);
                const double d0 = (bx * pq[0] + by * pq[1] - phi * pq[2]) * e +
                                  p * (bx * u[0] + by * u[1] - phi * u[2] - phi);
                s0 = fma(w, d0, s0);
            }
        }
    }
    if (dI0) dI0[pair * nn + node] = -s0;
    if (dI1) dI1[pair * nn + node] = -s1;
}

// ||G||^2 per pair (block partials, then the fixed-order finish)
__global__ void k_norm2_partials(const double* __restrict__ G, double* __restrict__ partials, int npart, int64_t nn3) {
    __shared__ double sh[NODE_THREADS / 64];
    const int pair = blockIdx.y;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn3; i += (int64_t)npart * blockDim.x) {
        const double v = G[pair * nn3 + i];
        acc = fma(v, v, acc);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[pair * npart + blockIdx.x] = s;
}

// A pair whose right-hand side is 0 has the solution 0: clear its iterate.
__global__ void k_zero_where_rhs_zero(double* __restrict__ U, const double* __restrict__ rhs_n2, int64_t nn3) {
    const int pair = blockIdx.y;
    if (rhs_n2[pair] != 0.0) return;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn3; i += (int64_t)gridDim.x * blockDim.x)
        U[pair * nn3 + i] = 0.0;
}

int launch_zero_where_rhs_zero(sf_context* c, double* U, const double* rhs_n2) {
    hipLaunchKernelGGL(k_zero_where_rhs_zero, dim3(c->npart, c->B), dim3(NODE_THREADS), 0, c->stream, U, rhs_n2,
                       3ll * c->W * c->H);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_norm2(sf_context* c, const double* G, double* out) {
    const int64_t nn3 = 3ll * c->W * c->H;
    hipLaunchKernelGGL(k_norm2_partials, dim3(c->npart, c->B), dim3(NODE_THREADS), 0, c->stream, G, c->partials,
                       c->npart, nn3);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize_norm, dim3(c->B), dim3(64), 0, c->stream, c->partials, c->npart, out);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_adjoint_gradients(sf_context* c, const double* U, const double* P, double* dI0, double* dI1,
                             double* dal) {
    const int64_t nn = (int64_t)c->W * c->H, ne = (int64_t)(c->W - 1) * (c->H - 1) * 2;
    if (dal) {
        hipLaunchKernelGGL(k_adj_alpha, dim3((unsigned)((ne + 255) / 256), c->B), dim3(256), 0, c->stream, U, P, dal,
                           c->W, c->H);
        SF_LAUNCH_CHECK();
    }
    if (dI0 || dI1) {
        hipLaunchKernelGGL(k_adj_frames, dim3((unsigned)((nn + 255) / 256), c->B), dim3(256), 0, c->stream, c->f0,
                           c->ft, U, P, dI0, dI1, c->W, c->H);
        SF_LAUNCH_CHECK();
    }
    return SF_OK;
}

// --- presmoothing (Section 1): f = K_sigma * I ------------------------------
// One pass of the separable Gaussian along x (axis 0) or y (axis 1): every
// output pixel sums w[k+R] in[clamped neighbour at offset k], k = -R..R in
// increasing order; B frames of W x H, row-major.
__global__ void k_blur(const double* __restrict__ in, double* __restrict__ out, const double* __restrict__ w,
                       int R, int W, int H, int64_t n, int axis) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t frame = i / ((int64_t)W * H);
    const int p = (int)(i - frame * W * H), x = p % W, y = p / W;
    const double* f = in + frame * W * H;
    double s = 0.0;
    for (int k = -R; k <= R; ++k) {
        const int xx = axis == 0 ? min(max(x + k, 0), W - 1) : x;
        const int yy = axis == 1 ? min(max(y + k, 0), H - 1) : y;
        s += w[k + R] * f[(int64_t)yy * W + xx];
    }
    out[i] = s;
}

// I -> smoothed frames in out (B frames), through tmp
int launch_presmooth(sf_context* c, const double* I, double* out, double* tmp) {
    const int64_t n = (int64_t)c->W * c->H * c->B;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_blur, dim3(blocks), dim3(256), 0, c->stream, I, tmp, c->blur_w, c->blur_r, c->W, c->H, n, 0);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_blur, dim3(blocks), dim3(256), 0, c->stream, tmp, out, c->blur_w, c->blur_r, c->W, c->H, n, 1);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_validate(sf_context* c, const double* I0, const double* I1, const double* alpha) {
    const int64_t nn = (int64_t)c->W * c->H * c->B;
    const int64_t ne = (int64_t)(c->W - 1) * (c->H - 1) * 2 * c->B;
    int blocks = (int)std::min<int64_t>((std::max(nn, ne) + 255) / 256, 4096);
    hipLaunchKernelGGL(k_validate, dim3(blocks), dim3(256), 0, c->stream, I0, I1, alpha, nn, ne, c->flags_d);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

static_assert(CLG_NCOEF == CLG_COEFS, "coefficient planes of the smoothed data term");

// K_rho data term: the coefficient planes of every element (two separable
// passes over the shifts), then F from them and ||F||^2.
int launch_clg(sf_context* c) {
    const int64_t ne = (int64_t)(c->W - 1) * (c->H - 1) * 2, nn = (int64_t)c->W * c->H;
    const unsigned eb = (unsigned)((ne + 255) / 256);
    hipLaunchKernelGGL(k_clg_smooth_x, dim3(eb, c->B), dim3(256), 0, c->stream, c->f0, c->ft, c->clg_w, c->clg_r,
                       c->clg_tmp, c->W, c->H);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_clg_smooth_y, dim3(eb, CLG_NCOEF, c->B), dim3(256), 0, c->stream, c->clg_tmp, c->clg_w,
                       c->clg_r, c->coef, c->W, c->H);
    SF_LAUNCH_CHECK();
    dim3 grid((unsigned)((nn + NODE_THREADS - 1) / NODE_THREADS), c->B);
    hipLaunchKernelGGL(k_clg_rhs, grid, dim3(NODE_THREADS), 0, c->stream, c->coef, c->alpha, c->F, c->partials,
                       c->npart, c->W, c->H);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize_norm, dim3(c->B), dim3(64), 0, c->stream, c->partials, c->npart, c->Fn2);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_assemble(sf_context* c, const double* I0, const double* I1, const double* alpha) {
    const int64_t nn = (int64_t)c->W * c->H;
    dim3 grid((unsigned)((nn + NODE_THREADS - 1) / NODE_THREADS), c->B);
    hipLaunchKernelGGL(k_assemble, grid, dim3(NODE_THREADS), 0, c->stream, I0, I1, alpha, c->f0, c->ft,
                       c->alpha, c->F, c->partials, c->npart, c->W, c->H);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize_norm, dim3(c->B), dim3(64), 0, c->stream, c->partials, c->npart, c->Fn2);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_residual(sf_context* c, const double* U, double* r, int fuse_converge, double rtol, int sweep,
                    int max_sweeps, const double* rhs, const double* rhs_n2) {
    if (!rhs) rhs = c->F;
    if (!rhs_n2) rhs_n2 = c->Fn2;
    const int64_t nn = (int64_t)c->W * c->H;
    dim3 grid((unsigned)((nn + NODE_THREADS - 1) / NODE_THREADS), c->B);
    const int32_t* done = fuse_converge ? (const int32_t*)c->done_d : (const int32_t*)nullptr;
    if (c->coef)
        hipLaunchKernelGGL(k_residual<true>, grid, dim3(NODE_THREADS), 0, c->stream, c->f0, c->alpha, rhs, U, r,
                           c->partials, c->npart, c->W, c->H, c->cfg.lambda, done, (const double*)c->coef);
    else
        hipLaunchKernelGGL(k_residual<false>, grid, dim3(NODE_THREADS), 0, c->stream, c->f0, c->alpha, rhs, U, r,
                           c->partials, c->npart, c->W, c->H, c->cfg.lambda, done, (const double*)nullptr);
    SF_LAUNCH_CHECK();
    if (fuse_converge) {
        hipLaunchKernelGGL(k_converge, dim3(c->B), dim3(NODE_THREADS), 0, c->stream, c->partials, c->npart,
                           rhs_n2, c->relres_d, c->sweeps_d, c->done_d, rtol, sweep, max_sweeps,
                           c->graph_capture ? (const int32_t*)c->gk_d : (const int32_t*)nullptr);
    } else {
        hipLaunchKernelGGL(k_finalize_norm, dim3(c->B), dim3(64), 0, c->stream, c->partials, c->npart,
                           c->relres_d);
    }
    SF_LAUNCH_CHECK();
    return SF_OK;
}

// ---- allocation-free residual (sf_residual_noalloc) ------------------------
//
// The block partials and the per-pair norms of the residual live in one
// file-scope device array instead of the context's arrays.  Every context on
// a device shares that device's copy, which keeps the last call's contents;
// nothing in it needs clearing (every block writes its partial, the finish
// kernel every norm).  Calls that overlap on one device race.
static __device__ __align__(256) double scratch[SF_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
double* scratch_addr[SCRATCH_MAX_DEVICES] = {};
}  // namespace

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.  The array's name in host code is a host-side stand-in,
// not a device address, so kernels and copies take this pointer.
int scratch_resolve(int device, double** out) {
    *out = nullptr;
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return SF_ERR_INVALID;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[device]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return SF_ERR_HIP;
        }
        scratch_addr[device] = (double*)p;
    }
    *out = scratch_addr[device];
    return SF_OK;
}

// Doubles of scratch the residual of a context needs: B blocks' partials of
// npart blocks each, then the B norms.
int64_t scratch_residual_doubles(const sf_context* c) { return (int64_t)c->B * c->npart + c->B; }

// r = F - A U with ||r||^2 per pair at scr + B npart; the same kernels, launch
// shape and reduction order as launch_residual, so r and the norms are equal
// bit for bit.
int launch_residual_scratch(sf_context* c, const double* U, double* r, double* scr) {
    const int64_t nn = (int64_t)c->W * c->H;
    dim3 grid((unsigned)((nn + NODE_THREADS - 1) / NODE_THREADS), c->B);
    if (c->coef)
        hipLaunchKernelGGL(k_residual<true>, grid, dim3(NODE_THREADS), 0, c->stream, c->f0, c->alpha, c->F, U, r,
                           scr, c->npart, c->W, c->H, c->cfg.lambda, (const int32_t*)nullptr, (const double*)c->coef);
    else
        hipLaunchKernelGGL(k_residual<false>, grid, dim3(NODE_THREADS), 0, c->stream, c->f0, c->alpha, c->F, U, r,
                           scr, c->npart, c->W, c->H, c->cfg.lambda, (const int32_t*)nullptr, (const double*)nullptr);
    SF_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_finalize_norm, dim3(c->B), dim3(64), 0, c->stream, scr, c->npart,
                       scr + (int64_t)c->B * c->npart);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_indicator(sf_context* c, const double* U, double* eta, int reset_max) {
    const int64_t ne = (int64_t)(c->W - 1) * (c->H - 1) * 2;
    if (reset_max) {
        hipLaunchKernelGGL(k_zero_u64, dim3((c->B + 255) / 256), dim3(256), 0, c->stream, c->etamax_bits, c->B);
        SF_LAUNCH_CHECK();
    }
    dim3 grid((unsigned)((ne + 255) / 256), c->B);
    hipLaunchKernelGGL(k_indicator, grid, dim3(256), 0, c->stream, c->f0, c->ft, c->alpha, U, eta,
                       c->etamax_bits, c->W, c->H, (const double*)c->coef);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

int launch_alpha_update(sf_context* c, const double* eta, double* alpha_out, double kappa, double eta_thr,
                        double alpha_th) {
    const int64_t ne = (int64_t)(c->W - 1) * (c->H - 1) * 2;
    dim3 grid((unsigned)((ne + 255) / 256), c->B);
    hipLaunchKernelGGL(k_alpha_update, grid, dim3(256), 0, c->stream, eta, c->etamax_bits, c->alpha, alpha_out,
                       ne, kappa, eta_thr, alpha_th);
    SF_LAUNCH_CHECK();
    return SF_OK;
}

}  // namespace sfdd

// Subdomain factorisation: block Cholesky of the banded subdomain matrix.
//
// Paper, Section 3.2: every subdomain problem is solved directly (the paper
// uses sparse LU from UMFPACK/MUMPS).  Ordered line by line along the shorter
// box side, A_i is block tridiagonal with m x m diagonal blocks A_tt and
// sparse couplings B_t = A[line t, line t-1] (each unknown couples to the
// straight and the diagonal neighbour node of the previous line, 6 entries);
// its band Cholesky factor is block bidiagonal.  Per line:
//     S_0 = A_00,   S_t = A_tt - B_t S_{t-1}^{-1} B_t^T
//     S_t = D_t D_t^T (Cholesky, pivots checked),   S_t^{-1} = D_t^{-T} D_t^{-1}
// and S_t^{-1} is stored as its lower-triangular 32x32 tiles, so a sweep
// applies each line with one symmetric matrix-vector product.
//
// Launch: one workgroup per subdomain; the m x m working matrices live in a
// per-subdomain workspace (L2-resident at the sizes used here).
#include <cmath>

#include <algorithm>

#include "element.h"
#include "sfdd_internal.h"

namespace sfdd {

// Lane-blocked 32x32x32 tile product for one wave:
//   acc[r][c] += sum_k opA(4br+r, k) * opB(k, 4bc+c),  br = lane/8, bc = lane%8
// opA(i,k) = TA ? A[k*lda+i] : A[i*lda+k];  opB(k,j) = TB ? B[j*ldb+k] : B[k*ldb+j].
template <bool TA, bool TB>
__device__ __forceinline__ void tile_mm(const double* A, int lda, const double* B, int ldb, double acc[4][4]) {
    const int lane = threadIdx.x & 63, br = lane >> 3, bc = lane & 7;
#pragma unroll 4
    for (int k = 0; k < TS; ++k) {
        double a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = TA ? A[k * lda + 4 * br + r] : A[(4 * br + r) * lda + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = TB ? B[(4 * bc + c) * ldb + k] : B[k * ldb + 4 * bc + c];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = fma(a[r], b[c], acc[r][c]);
    }
}

__device__ __forceinline__ void acc_zero(double acc[4][4]) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;
}

__device__ __forceinline__ void acc_load(double acc[4][4], const double* C, int ldc) {
    const int lane = threadIdx.x & 63, br = lane >> 3, bc = lane & 7;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = C[(4 * br + r) * ldc + 4 * bc + c];
}

__device__ __forceinline__ void acc_store(const double acc[4][4], double* C, int ldc, double scale = 1.0) {
    const int lane = threadIdx.x & 63, br = lane >> 3, bc = lane & 7;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) C[(4 * br + r) * ldc + 4 * bc + c] = scale * acc[r][c];
}

// the same into a tile of single-precision storage (each value rounded once)
__device__ __forceinline__ void acc_store_f(const double acc[4][4], float* C, int ldc) {
    const int lane = threadIdx.x & 63, br = lane >> 3, bc = lane & 7;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) C[(4 * br + r) * ldc + 4 * bc + c] = (float)acc[r][c];
}

__device__ __forceinline__ void acc_store_t(const double acc[4][4], double* C, int ldc) {
    const int lane = threadIdx.x & 63, br = lane >> 3, bc = lane & 7;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) C[(4 * bc + c) * ldc + 4 * br + r] = acc[r][c];
}

__device__ void set_status(DevStatus* st, int code, int sub, int64_t row) {
    if (atomicCAS(&st->code, 0, code) == 0) {
        st->sub = sub;
        st->row = row;
    }
}

__global__ void __launch_bounds__(FACTOR_THREADS)
k_factor(const SubDesc* __restrict__ subs, const double* __restrict__ f0_all, const double* __restrict__ al_all,
         double* __restrict__ factors, double* __restrict__ work, DevStatus* __restrict__ status,
         int W, int H, double lam, int fp32, int sub0, const double* __restrict__ coef_all) {
    const int sub = sub0 + blockIdx.x;
    const SubDesc d = subs[sub];
    const int tid = threadIdx.x, wv = tid >> 6, nw = FACTOR_THREADS / 64;
    const int m = d.m, mp = d.mp, NT = d.NT, ms = d.ms;
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const double* f0 = f0_all + d.pair * nn;
    const double* al = al_all + d.pair * ne;
    const double* cf = coef_all ? coef_all + (int64_t)d.pair * CLG_NCOEF * ne : nullptr;   // K_rho data term
    double* S = work + d.soff;                 // mp x mp: S_t, then its Cholesky factor
    double* Y = S + (int64_t)mp * mp;          // mp x mp: B P, then D^{-1}
    double* Pv = Y + (int64_t)mp * mp;         // mp x mp: S_{t-1}^{-1}, full symmetric
    double* Tout = factors + d.foff;
    double* Bst = factors + d.boff;

    __shared__ double sh_tile[TSZ];            // diagonal tile being factored
    __shared__ double sh_inv[TSZ];             // its inverse
    __shared__ double sh_acc[4][TSZ];          // per-wave tile scratch
    __shared__ double sh_dg[512];              // diagonal of S_t before factoring
    __shared__ int sh_fail;

    if (tid == 0) sh_fail = 0;
    for (int t = 0; t < d.nt; ++t) {
        // ---- 0. A_tt and B_t from the stencil --------------------------------
        for (int64_t i = tid; i < (int64_t)mp * mp; i += FACTOR_THREADS) {
            const int a = (int)(i / mp), b = (int)(i % mp);
            S[i] = (a == b && a >= m) ? 1.0 : 0.0;
        }
        __syncthreads();
        for (int s = tid; s < ms; s += FACTOR_THREADS) {
            int x, y;
            local_to_global(d, t, s, x, y);
            double blk[9];
            stencil_block(f0, al, W, H, x, y, 0, 0, lam, blk, cf);
            for (int c = 0; c < 3; ++c)
                for (int e = 0; e < 3; ++e) S[(3 * s + c) * mp + 3 * s + e] = blk[3 * c + e];
            if (s + 1 < ms) {   // next node along the line
                if (d.cols) stencil_block(f0, al, W, H, x, y, 0, 1, lam, blk, cf);
                else        stencil_block(f0, al, W, H, x, y, 1, 0, lam, blk, cf);
                for (int c = 0; c < 3; ++c)
                    for (int e = 0; e < 3; ++e) {
                        S[(3 * s + c) * mp + 3 * (s + 1) + e] = blk[3 * c + e];
                        S[(3 * (s + 1) + e) * mp + 3 * s + c] = blk[3 * c + e];
                    }
            }
            if (t > 0) {
                // couplings to the previous line: straight neighbour (same s) and
                // diagonal neighbour (s - 1); both are "previous" nodes, so take the
                // positive-direction block from them and transpose.
                int px, py;
                local_to_global(d, t - 1, s, px, py);
                double bs[9], bd[9];
                if (d.cols) stencil_block(f0, al, W, H, px, py, 1, 0, lam, bs, cf);
                else        stencil_block(f0, al, W, H, px, py, 0, 1, lam, bs, cf);
                if (s > 0) {
                    int qx, qy;
                    local_to_global(d, t - 1, s - 1, qx, qy);
                    stencil_block(f0, al, W, H, qx, qy, 1, 1, lam, bd, cf);
                } else {
                    for (int k = 0; k < 9; ++k) bd[k] = 0.0;
                }
                double* row = Bst + ((int64_t)t * m + 3 * s) * 6;
                for (int c = 0; c < 3; ++c)
                    for (int e = 0; e < 3; ++e) {
                        row[c * 6 + e] = bd[3 * e + c];       // B[3s+c][3(s-1)+e]
                        row[c * 6 + 3 + e] = bs[3 * e + c];   // B[3s+c][3s+e]
                    }
            }
        }
        __syncthreads();
        // ---- 1. S_t -= B_t P B_t^T ------------------------------------------
        if (t > 0) {
            const double* Bt = Bst + (int64_t)t * m * 6;
            for (int64_t i = tid; i < (int64_t)m * m; i += FACTOR_THREADS) {
                const int a = (int)(i / m), b2 = (int)(i % m);
                const int s = a / 3;
                const double* cf = Bt + (int64_t)a * 6;
                double v = 0.0;
                for (int e = 0; e < 3; ++e) {
                    if (s > 0) v = fma(cf[e], Pv[(int64_t)(3 * (s - 1) + e) * mp + b2], v);
                    v = fma(cf[3 + e], Pv[(int64_t)(3 * s + e) * mp + b2], v);
                }
                Y[(int64_t)a * mp + b2] = v;
            }
            __syncthreads();
            for (int64_t i = tid; i < (int64_t)m * m; i += FACTOR_THREADS) {
                const int a = (int)(i / m), a2 = (int)(i % m);
                const int s2 = a2 / 3;
                const double* cf = Bt + (int64_t)a2 * 6;
                double v = 0.0;
                for (int e = 0; e < 3; ++e) {
                    if (s2 > 0) v = fma(Y[(int64_t)a * mp + 3 * (s2 - 1) + e], cf[e], v);
                    v = fma(Y[(int64_t)a * mp + 3 * s2 + e], cf[3 + e], v);
                }
                S[(int64_t)a * mp + a2] -= v;
            }
            __syncthreads();
        }
        for (int a = tid; a < mp; a += FACTOR_THREADS) sh_dg[a] = S[(int64_t)a * mp + a];
        __syncthreads();
        // ---- 2. blocked right-looking Cholesky -------------------------------
        for (int k = 0; k < NT; ++k) {
            double* Skk = S + (int64_t)(k * TS) * mp + k * TS;
            for (int i = tid; i < TSZ; i += FACTOR_THREADS) sh_tile[i] = Skk[(i / TS) * mp + (i % TS)];
            __syncthreads();
            for (int j = 0; j < TS; ++j) {
                if (tid == 0) {
                    const double piv = sh_tile[j * TS + j];
                    const double ref = sh_dg[k * TS + j];
                    if (!(piv > 1e-13 * ref) || !isfinite(piv)) {
                        if (!sh_fail) set_status(status, SF_NOT_SPD, sub, (int64_t)t * m + k * TS + j);
                        sh_fail = 1;
                        sh_tile[j * TS + j] = 1.0;
                    } else {
                        sh_tile[j * TS + j] = sqrt(piv);
                    }
                }
                __syncthreads();
                const double djj = sh_tile[j * TS + j];
                if (tid > j && tid < TS) sh_tile[tid * TS + j] /= djj;
                __syncthreads();
                for (int i = tid; i < TSZ; i += FACTOR_THREADS) {
                    const int r = i / TS, c = i % TS;
                    if (c > j && r >= c) sh_tile[i] -= sh_tile[r * TS + j] * sh_tile[c * TS + j];
                }
                __syncthreads();
            }
            // inverse of the diagonal factor tile (lower triangular), column per thread
            if (tid < TS) {
                const int j = tid;
                for (int i = 0; i < TS; ++i) sh_inv[i * TS + j] = 0.0;
                for (int i = j; i < TS; ++i) {
                    double s = (i == j) ? 1.0 : 0.0;
                    for (int q = j; q < i; ++q) s -= sh_tile[i * TS + q] * sh_inv[q * TS + j];
                    sh_inv[i * TS + j] = s / sh_tile[i * TS + i];
                }
            }
            __syncthreads();
            for (int i = tid; i < TSZ; i += FACTOR_THREADS) {
                const int r = i / TS, c = i % TS;
                Skk[r * mp + c] = (c <= r) ? sh_tile[i] : 0.0;
                Y[(int64_t)(k * TS + r) * mp + k * TS + c] = sh_inv[i];
            }
            __syncthreads();
            // panel: L_ik = S_ik D_kk^{-T}
            for (int i = k + 1 + wv; i < NT; i += nw) {
                double acc[4][4];
                acc_zero(acc);
                double* Sik = S + (int64_t)(i * TS) * mp + k * TS;
                tile_mm<false, true>(Sik, mp, sh_inv, TS, acc);
                acc_store(acc, Sik, mp);
            }
            __syncthreads();
            // trailing update: S_ij -= L_ik L_jk^T, k < j <= i
            const int nrem = NT - k - 1;
            const int npairs = nrem * (nrem + 1) / 2;
            for (int q = wv; q < npairs; q += nw) {
                int ii = 0;
                while ((ii + 1) * (ii + 2) / 2 <= q) ++ii;
                const int jj = q - ii * (ii + 1) / 2;
                const int i = k + 1 + ii, j = k + 1 + jj;
                double acc[4][4];
                double* Sij = S + (int64_t)(i * TS) * mp + j * TS;
                acc_load(acc, Sij, mp);
                double neg[4][4];
                acc_zero(neg);
                tile_mm<false, true>(S + (int64_t)(i * TS) * mp + k * TS, mp, S + (int64_t)(j * TS) * mp + k * TS, mp, neg);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int c = 0; c < 4; ++c) acc[r][c] -= neg[r][c];
                acc_store(acc, Sij, mp);
            }
            __syncthreads();
        }
        // ---- 3. D^{-1} (lower, into Y), one block row at a time -------------
        //   D^{-1}_ij = -D_ii^{-1} sum_{k=j}^{i-1} L_ik D^{-1}_kj,  j < i
        for (int i = 1; i < NT; ++i) {
            for (int jb = 0; jb < i; jb += nw) {
                const int j = jb + wv;
                const bool act = j < i;
                double acc[4][4];
                acc_zero(acc);
                if (act) {
                    for (int k = j; k < i; ++k)
                        tile_mm<false, false>(S + (int64_t)(i * TS) * mp + k * TS, mp,
                                              Y + (int64_t)(k * TS) * mp + j * TS, mp, acc);
                    acc_store(acc, sh_acc[wv], TS);
                }
                __syncthreads();
                if (act) {
                    double out[4][4];
                    acc_zero(out);
                    tile_mm<false, false>(Y + (int64_t)(i * TS) * mp + i * TS, mp, sh_acc[wv], TS, out);
                    acc_store(out, Y + (int64_t)(i * TS) * mp + j * TS, mp, -1.0);
                }
                __syncthreads();
            }
        }
        // ---- 4. S^{-1} = D^{-T} D^{-1}: lower tiles out, full copy for the next line
        const int ntl = NT * (NT + 1) / 2;
        for (int q = wv; q < ntl; q += nw) {
            int i = 0;
            while ((i + 1) * (i + 2) / 2 <= q) ++i;
            const int j = q - i * (i + 1) / 2;
            double acc[4][4];
            acc_zero(acc);
            for (int k = i; k < NT; ++k)
                tile_mm<true, false>(Y + (int64_t)(k * TS) * mp + i * TS, mp, Y + (int64_t)(k * TS) * mp + j * TS, mp, acc);
            if (fp32) acc_store_f(acc, reinterpret_cast<float*>(Tout) + ((int64_t)t * d.ntiles + q) * TSZ, TS);
            else      acc_store(acc, Tout + ((int64_t)t * d.ntiles + q) * TSZ, TS);
            acc_store(acc, Pv + (int64_t)(i * TS) * mp + j * TS, mp);
            if (i != j) acc_store_t(acc, Pv + (int64_t)(j * TS) * mp + i * TS, mp);
        }
        __syncthreads();
    }
}

__global__ void k_zero_status(DevStatus* st) {
    st->code = 0;
    st->sub = -1;
    st->row = -1;
}

int launch_factor(sf_context* c) {
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(1), 0, c->stream, c->status_d);
    if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
    // chunks of subdomains that share the factor workspace slots, in order
    for (int s0 = 0; s0 < c->nsub; s0 += c->factor_chunk) {
        const int n = std::min(c->factor_chunk, c->nsub - s0);
        hipLaunchKernelGGL(k_factor, dim3(n), dim3(FACTOR_THREADS), 0, c->stream, c->d_subs, c->f0, c->alpha,
                           c->factors, c->work, c->status_d, c->W, c->H, c->cfg.lambda,
                           c->cfg.factor_precision != SF_FP64 ? 1 : 0, s0, (const double*)c->coef);
        if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace sfdd

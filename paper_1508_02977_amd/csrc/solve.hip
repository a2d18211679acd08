// Restricted additive Schwarz sweep (paper, Section 4.2, equation (schwarz)).
//
// For every subdomain i (all pairs at once): e_i = A_i^{-1} r[S_i] and
// U[O_i] += e_i[O_i], where r = F - A U of the current iterate.  With the
// block factorisation of factor.hip (line couplings B_t, inverted Schur
// complements S_t^{-1}) the local solve is
//     forward:  z_0 = r_0,  w_t = S_t^{-1} z_t,  z_{t+1} = r_{t+1} - B_{t+1} w_t
//     backward: x_{nt-1} = w_{nt-1},  x_t = w_t - S_t^{-1} (B_{t+1}^T x_{t+1})
// i.e. one dense symmetric matrix-vector product per line and direction.
//
// Parallel layout: P workgroups cooperate on one subdomain.  Each holds a
// fixed share of the 32x32 lower tiles of every S_t^{-1} (tile k of a line
// goes to rank k mod P) and streams them once per direction; an off-diagonal
// tile contributes T z_J to rows I and T^T z_I to rows J.  Ranks publish
// partial result vectors and bump a per-subdomain counter; at the next line
// every rank sums the P partials in rank order (bitwise reproducible).  All
// waits are bounded: a stalled wait raises SF_ERR_DEVICE and every rank exits.
#include "sfdd_internal.h"

namespace sfdd {

constexpr int MAXMP = 512;

struct SweepArgs {
    const SubDesc* subs;
    const int32_t* wgmap;
    const double* factors;
    double* work;
    const double* r;        // global residual [B][3][H][W] (mode 0)
    double* U;              // global iterate (mode 0)
    const int32_t* done;    // [B] converged pairs (mode 0)
    const double* b_local;  // local right-hand side (mode 1)
    double* x_local;        // local solution (mode 1)
    uint32_t* counters;
    DevStatus* status;
    int W, H, mode;
    long long spin_limit;
};

__device__ __forceinline__ bool wait_count(uint32_t* cnt, uint32_t target, const SweepArgs& A, int sub,
                                           int* sh_ok) {
    if (threadIdx.x == 0) {
        long long n = 0;
        int ok = 1;
        while (__hip_atomic_load(cnt, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(&A.status->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SF_ERR_DEVICE ||
                ++n > A.spin_limit) {
                if (atomicCAS(&A.status->code, 0, SF_ERR_DEVICE) == 0) {
                    A.status->sub = sub;
                    A.status->row = (int64_t)target;
                }
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        *sh_ok = ok;
    }
    __syncthreads();
    return *sh_ok != 0;
}

__device__ __forceinline__ void signal_count(uint32_t* cnt) {
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Contribution of this rank's tiles of one line matrix to y = S^{-1} z.
// z and the per-wave accumulators yw[4][mp] live in LDS.
__device__ __forceinline__ void apply_tiles(const double* __restrict__ Tl, int ntiles, int rank, int P,
                                            const double* z, double (*yw)[MAXMP]) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int j = lane & 31, h = lane >> 5;
    double* y = yw[wv];
    int idx = 0;
    for (int k = rank; k < ntiles; k += P, ++idx) {
        if ((idx & 3) != wv) continue;
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= k) ++I;
        const int J = k - I * (I + 1) / 2;
        const double* T = Tl + (int64_t)k * TSZ + (16 * h) * TS + j;
        double tv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) tv[i] = T[i * TS];
        // y_J += T^T z_I  (for a diagonal tile this is the whole product)
        const double* zI = z + I * TS + 16 * h;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) s = fma(tv[i], zI[i], s);
        s += __shfl_xor(s, 32, 64);
        if (h == 0) y[J * TS + j] += s;
        if (I != J) {
            // y_I += T z_J: per lane 16 row products, reduced over the 32 lanes of
            // the half by a transpose-reduce butterfly (xor 16, 8, 4, 2, then 1).
            const double zj = z[J * TS + j];
            double p[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) p[i] = tv[i] * zj;
            const int b4 = (j >> 4) & 1, b3 = (j >> 3) & 1, b2 = (j >> 2) & 1, b1 = (j >> 1) & 1;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const double keep = b4 ? p[q + 8] : p[q], send = b4 ? p[q] : p[q + 8];
                p[q] = keep + __shfl_xor(send, 16, 64);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double keep = b3 ? p[q + 4] : p[q], send = b3 ? p[q] : p[q + 4];
                p[q] = keep + __shfl_xor(send, 8, 64);
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const double keep = b2 ? p[q + 2] : p[q], send = b2 ? p[q] : p[q + 2];
                p[q] = keep + __shfl_xor(send, 4, 64);
            }
            {
                const double keep = b1 ? p[1] : p[0], send = b1 ? p[0] : p[1];
                p[0] = keep + __shfl_xor(send, 2, 64);
            }
            p[0] += __shfl_xor(p[0], 1, 64);
            if ((j & 1) == 0) {
                const int row = 8 * b4 + 4 * b3 + 2 * b2 + b1;
                y[I * TS + 16 * h + row] += p[0];
            }
        }
    }
}

__global__ void __launch_bounds__(SOLVE_THREADS) k_sweep(SweepArgs A) {
    __shared__ double z[MAXMP];
    __shared__ double full[MAXMP];
    __shared__ double yw[4][MAXMP];
    __shared__ int sh_ok;

    const int code = A.wgmap[blockIdx.x];
    const int sub = code >> 8, rank = code & 255;
    const SubDesc d = A.subs[sub];
    if (A.mode == 0 && A.done[d.pair]) return;   // uniform over the subdomain's ranks
    const int tid = threadIdx.x;
    const int P = d.P, m = d.m, mp = d.mp, ms = d.ms, nt = d.nt, ntiles = d.ntiles;
    const int64_t nn = (int64_t)A.W * A.H;
    const double* Tb = A.factors + d.foff;
    const double* Bb = A.factors + d.boff;
    double* wst = A.work + d.woff;
    double* part = A.work + d.poff;          // [2][P][mp]
    uint32_t* cnt = A.counters + sub;
    const int sl0 = (rank * mp) / P, sl1 = ((rank + 1) * mp) / P;   // this rank's slice

    auto rhs = [&](int t, int a) -> double {
        if (A.mode == 1) return A.b_local[(int64_t)t * m + a];
        int x, y;
        local_to_global(d, t, a / 3, x, y);
        return A.r[((int64_t)d.pair * 3 + a % 3) * nn + (int64_t)y * A.W + x];
    };
    auto emit = [&](int t, int a, double v) {
        if (A.mode == 1) { A.x_local[(int64_t)t * m + a] = v; return; }
        int x, y;
        local_to_global(d, t, a / 3, x, y);
        if (x >= d.ox0 && x < d.ox1 && y >= d.oy0 && y < d.oy1)
            A.U[((int64_t)d.pair * 3 + a % 3) * nn + (int64_t)y * A.W + x] += v;
    };
    // full <- base - sum_q part[buf][q]  (base may be null: +sum)
    auto gather = [&](int buf, const double* base) {
        const double* pb = part + (int64_t)buf * P * mp;
        for (int a = tid; a < mp; a += SOLVE_THREADS) {
            double s = 0.0;
            for (int q = 0; q < P; ++q) s += pb[(int64_t)q * mp + a];
            full[a] = base ? base[a] - s : s;
        }
    };
    auto publish = [&](int buf) {
        double* pb = part + ((int64_t)buf * P + rank) * mp;
        for (int a = tid; a < mp; a += SOLVE_THREADS) pb[a] = yw[0][a] + yw[1][a] + yw[2][a] + yw[3][a];
    };
    auto clear_y = [&]() {
        for (int a = tid; a < mp; a += SOLVE_THREADS) {
            yw[0][a] = 0.0; yw[1][a] = 0.0; yw[2][a] = 0.0; yw[3][a] = 0.0;
        }
    };

    uint32_t phase = 0;
    // ---------------- forward ----------------
    for (int t = 0; t < nt; ++t, ++phase) {
        if (t > 0) {
            if (!wait_count(cnt, P * phase, A, sub, &sh_ok)) return;
            gather((phase - 1) & 1, nullptr);          // full = w_{t-1}
            __syncthreads();
            for (int a = sl0 + tid; a < sl1; a += SOLVE_THREADS) wst[(int64_t)(t - 1) * mp + a] = full[a];
        }
        const double* Bt = Bb + (int64_t)t * m * 6;
        for (int a = tid; a < mp; a += SOLVE_THREADS) {
            double v = 0.0;
            if (a < m) {
                v = rhs(t, a);
                if (t > 0) {
                    const int s = a / 3;
                    const double* cf = Bt + (int64_t)a * 6;
                    double bw = 0.0;
                    if (s > 0)
                        for (int e = 0; e < 3; ++e) bw = fma(cf[e], full[3 * (s - 1) + e], bw);
                    for (int e = 0; e < 3; ++e) bw = fma(cf[3 + e], full[3 * s + e], bw);
                    v -= bw;
                }
            }
            z[a] = v;
        }
        clear_y();
        __syncthreads();
        apply_tiles(Tb + (int64_t)t * ntiles * TSZ, ntiles, rank, P, z, yw);
        __syncthreads();
        publish(phase & 1);
        signal_count(cnt);
    }
    // ---------------- backward ----------------
    for (int t = nt - 2; t >= 0; --t, ++phase) {
        if (!wait_count(cnt, P * phase, A, sub, &sh_ok)) return;
        // full = x_{t+1}
        gather((phase - 1) & 1, (t + 1 == nt - 1) ? nullptr : wst + (int64_t)(t + 1) * mp);
        __syncthreads();
        for (int a = sl0 + tid; a < sl1; a += SOLVE_THREADS)
            if (a < m) emit(t + 1, a, full[a]);
        // z = B_{t+1}^T x_{t+1}
        const double* Bt = Bb + (int64_t)(t + 1) * m * 6;
        for (int b = tid; b < mp; b += SOLVE_THREADS) {
            double v = 0.0;
            if (b < m) {
                const int s = b / 3, e = b % 3;
                for (int c = 0; c < 3; ++c) v = fma(Bt[(int64_t)(3 * s + c) * 6 + 3 + e], full[3 * s + c], v);
                if (s + 1 < ms)
                    for (int c = 0; c < 3; ++c)
                        v = fma(Bt[(int64_t)(3 * (s + 1) + c) * 6 + e], full[3 * (s + 1) + c], v);
            }
            z[b] = v;
        }
        clear_y();
        __syncthreads();
        apply_tiles(Tb + (int64_t)t * ntiles * TSZ, ntiles, rank, P, z, yw);
        __syncthreads();
        publish(phase & 1);
        signal_count(cnt);
    }
    // x_0
    if (!wait_count(cnt, P * phase, A, sub, &sh_ok)) return;
    gather((phase - 1) & 1, nt == 1 ? nullptr : wst);
    __syncthreads();
    for (int a = sl0 + tid; a < sl1; a += SOLVE_THREADS)
        if (a < m) emit(0, a, full[a]);
}

__global__ void k_zero_u32(uint32_t* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

const void* sweep_kernel() { return (const void*)k_sweep; }

int launch_sweep(sf_context* c, double* U, const double* r, int single_sub, const double* b_local, double* x_local) {
    SweepArgs a;
    a.subs = c->d_subs;
    a.wgmap = c->d_wgmap;
    a.factors = c->factors;
    a.work = c->work;
    a.r = r;
    a.U = U;
    a.done = c->done_d;
    a.b_local = b_local;
    a.x_local = x_local;
    a.counters = c->counters;
    a.status = c->status_d;
    a.W = c->W;
    a.H = c->H;
    a.mode = single_sub >= 0 ? 1 : 0;
    a.spin_limit = 1ll << 20;
    int grid = c->sweep_grid;
    if (single_sub >= 0) {
        hipLaunchKernelGGL(k_zero_u32, dim3((c->nsub + 255) / 256), dim3(256), 0, c->stream, c->counters, c->nsub);
        if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
        // second half of the map: subdomain-major order
        a.wgmap = c->d_wgmap + (int64_t)c->nsub * c->maxP + (int64_t)single_sub * c->maxP;
        grid = c->maxP;
    }
    if (c->maxP > 1) {
        void* args[] = {&a};
        if (hipLaunchCooperativeKernel((const void*)k_sweep, dim3(grid), dim3(SOLVE_THREADS), args, 0, c->stream) !=
            hipSuccess)
            return SF_ERR_HIP;
    } else {
        hipLaunchKernelGGL(k_sweep, dim3(grid), dim3(SOLVE_THREADS), 0, c->stream, a);
        if (hipGetLastError() != hipSuccess) return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace sfdd

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
// Parallel layout: P workgroups (ranks) cooperate on one subdomain.  Rank p
// computes the block rows I = p, p+P, ... of every product S_t^{-1} z: the
// tiles of block row I are the lower tiles (I, J<=I) and, transposed, the
// tiles (J>I, I) of block column I, so each off-diagonal tile is read by two
// ranks (the second read is served by L2: all ranks of a subdomain sit on one
// XCD).  Ranks publish their finished rows and bump a per-subdomain counter;
// the next line starts when all P rows sets are out.  No reductions across
// ranks, so results do not depend on P.  All waits are bounded: a stalled
// wait raises SF_ERR_DEVICE and every rank exits.
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

// Thread 0 polls the counter with relaxed device-scope loads (they bypass the
// non-coherent caches); the other waves wait at the barrier.  Bounded: on a
// stall the wait records SF_ERR_DEVICE and every rank of every subdomain exits.
__device__ __forceinline__ bool wait_count(uint32_t* cnt, uint32_t target, const SweepArgs& A, int sub,
                                           int* sh_ok) {
    if (threadIdx.x == 0) {
        long long n = 0;
        int ok = 1;
        while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
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

// Every value another rank reads is stored with a relaxed device-scope atomic
// (written through to the coherence point); waiting for all of them to be
// acknowledged before the counter increment orders data before flag without
// a cache-wide writeback.
__device__ __forceinline__ void signal_count(uint32_t* cnt) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void pub_store(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double pub_load(const double* p) {
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Rows I*32 .. I*32+31 of y = S z for the symmetric line matrix S stored as
// its lower 32x32 tiles (tile (I,J), I >= J, at index I(I+1)/2 + J):
//   y_I = sum_{J <= I} T(I,J) z_J + sum_{J > I} T(J,I)^T z_J.
// A wave takes tiles j0, j0+nwaves, ... of the NT tiles of the block row and
// accumulates into its own LDS row buffer yw[32].
__device__ __forceinline__ void block_row(const double* __restrict__ Tl, int NT, int I, const double* z,
                                          double* yw, int wv, int nwaves) {
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, h = lane >> 5;
    for (int J = wv; J < NT; J += nwaves) {
        const bool lower = J <= I;
        const int k = lower ? I * (I + 1) / 2 + J : J * (J + 1) / 2 + I;
        const double* T = Tl + (int64_t)k * TSZ + (16 * h) * TS + j;
        double tv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) tv[i] = T[i * TS];
        if (!lower || J == I) {
            // y_I[j] += sum_r T[r][j] zJ[r]: T = T(J,I) (transposed use) or the
            // symmetric diagonal tile; rows r of this lane are 16h..16h+15
            const double* zr = z + J * TS + 16 * h;
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 16; ++i) s = fma(tv[i], zr[i], s);
            s += __shfl_xor(s, 32, 64);
            if (h == 0) yw[j] += s;
        } else {
            // y_I[r] += sum_j T[r][j] zJ[j]: 16 row products per lane reduced over
            // the 32 lanes of the half (transpose-reduce: xor 16, 8, 4, 2, then 1)
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
            if ((j & 1) == 0) yw[16 * h + 8 * b4 + 4 * b3 + 2 * b2 + b1] += p[0];
        }
    }
}

__global__ void __launch_bounds__(SOLVE_THREADS) k_sweep(SweepArgs A) {
    constexpr int NW = SOLVE_THREADS / 64;
    __shared__ double z[MAXMP];
    __shared__ double full[MAXMP];
    __shared__ double yw[NW][TS];
    __shared__ int sh_ok;

    const int code = A.wgmap[blockIdx.x];
    const int sub = code >> 8, rank = code & 255;
    const SubDesc d = A.subs[sub];
    if (A.mode == 0 && A.done[d.pair]) return;   // uniform over the subdomain's ranks
    const int tid = threadIdx.x, wv = tid >> 6;
    const int P = d.P, m = d.m, mp = d.mp, ms = d.ms, nt = d.nt, ntiles = d.ntiles, NT = d.NT;
    const int64_t nn = (int64_t)A.W * A.H;
    const double* Tb = A.factors + d.foff;
    const double* Bb = A.factors + d.boff;
    double* wst = A.work + d.woff;           // forward results of this rank's rows
    double* pub = A.work + d.poff;           // [2][mp] published rows (double-buffered)
    uint32_t* cnt = A.counters + sub;

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
    // This rank's block rows I = rank, rank + P, ...: y = S_t z for those rows,
    // then finish(I, row, y) for each row.
    auto rows = [&](int t, auto&& finish) {
        const double* Tl = Tb + (int64_t)t * ntiles * TSZ;
        for (int I = rank; I < NT; I += P) {
            for (int i = tid; i < NW * TS; i += SOLVE_THREADS) (&yw[0][0])[i] = 0.0;
            __syncthreads();
            block_row(Tl, NT, I, z, yw[wv], wv, NW);
            __syncthreads();
            if (tid < TS) {
                double y = 0.0;
                for (int w = 0; w < NW; ++w) y += yw[w][tid];
                finish(I * TS + tid, y);
            }
            __syncthreads();
        }
    };

    uint32_t phase = 0;
    // ---------------- forward: w_t = S_t^{-1} (r_t - B_t w_{t-1}) ----------------
    for (int t = 0; t < nt; ++t, ++phase) {
        if (t > 0) {
            if (!wait_count(cnt, P * phase, A, sub, &sh_ok)) return;
            const double* pb = pub + (int64_t)((phase - 1) & 1) * mp;
            for (int a = tid; a < mp; a += SOLVE_THREADS) full[a] = pub_load(pb + a);
            __syncthreads();
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
        __syncthreads();
        double* pw = pub + (int64_t)(phase & 1) * mp;
        rows(t, [&](int a, double y) {
            pub_store(pw + a, y);
            wst[(int64_t)t * mp + a] = y;
            if (t == nt - 1 && a < m) emit(t, a, y);      // x_{nt-1} = w_{nt-1}
        });
        signal_count(cnt);
    }
    // ---------------- backward: x_t = w_t - S_t^{-1} B_{t+1}^T x_{t+1} ----------------
    for (int t = nt - 2; t >= 0; --t, ++phase) {
        if (!wait_count(cnt, P * phase, A, sub, &sh_ok)) return;
        const double* pb = pub + (int64_t)((phase - 1) & 1) * mp;
        for (int a = tid; a < mp; a += SOLVE_THREADS) full[a] = pub_load(pb + a);   // x_{t+1}
        __syncthreads();
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
        __syncthreads();
        double* pw = pub + (int64_t)(phase & 1) * mp;
        rows(t, [&](int a, double y) {
            const double x = wst[(int64_t)t * mp + a] - y;
            pub_store(pw + a, x);
            if (a < m) emit(t, a, x);
        });
        signal_count(cnt);
    }
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

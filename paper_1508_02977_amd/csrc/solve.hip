// Restricted additive Schwarz sweep (paper, Section 3.2, equation (schwarz)).
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
#include <algorithm>

#include "sfdd_internal.h"

namespace sfdd {

constexpr int MAXMP = 512;

struct SweepArgs {
    const SubDesc* subs;
    int nsub;               // subdomains (mode 0) ; the single subdomain index (mode 1)
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
    uint32_t epoch;         // tag base of this launch (published words carry epoch + phase)
    long long spin_limit;
};

constexpr int MAXR = 16;   // block rows per rank (NT <= 16)
constexpr int PF = 2;      // tiles per wave held in registers across the wait

// Tile (I, J) of the block row of symmetric S: lower tile (I,J) if J <= I,
// else the lower tile (J,I) used transposed.  Lane (j, h) holds column j of
// rows 16h..16h+15 of the stored tile.
__device__ __forceinline__ void load_tile(const double* __restrict__ Tl, int I, int J, double tv[16]) {
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, h = lane >> 5;
    const int k = J <= I ? I * (I + 1) / 2 + J : J * (J + 1) / 2 + I;
    const double* T = Tl + (int64_t)k * TSZ + (16 * h) * TS + j;
#pragma unroll
    for (int i = 0; i < 16; ++i) tv[i] = T[i * TS];
}

// y_I += (tile) z_J for one tile of the block row, into the wave's row buffer y[32].
__device__ __forceinline__ void tile_apply(const double tv[16], int I, int J, const double* z, double* y) {
    const int lane = threadIdx.x & 63;
    const int j = lane & 31, h = lane >> 5;
    if (J >= I) {
        // stored (J, I) used transposed, or the symmetric diagonal tile:
        // y_I[j] += sum_r T[r][j] zJ[r], rows r = 16h..16h+15 of this lane
        const double* zr = z + J * TS + 16 * h;
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 16; ++i) s = fma(tv[i], zr[i], s);
        s += __shfl_xor(s, 32, 64);
        if (h == 0) y[j] += s;
    } else {
        // stored (I, J): y_I[r] += sum_j T[r][j] zJ[j]; 16 row products per lane
        // reduced over the 32 lanes of the half (transpose-reduce: xor 16, 8, 4, 2, then 1)
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
        if ((j & 1) == 0) y[16 * h + 8 * b4 + 4 * b3 + 2 * b2 + b1] += p[0];
    }
}

// Phase q of a sweep: forward lines 0..nt-1, then backward lines nt-2..0.
// Waves 0..NW-2 ("tile waves") hold this rank's tiles of the line matrix and
// the right-hand side terms; the last wave ("control wave") does all the
// latency-critical traffic: it polls the counter, gathers the published rows,
// finishes and publishes this rank's rows and signals.  Global loads of a wave
// complete in order, so keeping the large tile prefetch (issued by the tile
// waves right after their compute, one phase ahead) off the control wave lets
// the next phase's data stream in while the control wave synchronises.  All
// addressing is set up once in registers; nothing inside the phase loop loads
// an address from memory (such a load would drain the prefetch queue).
// Workgroup g is dispatched to XCD g % 8; the ranks of subdomain i are the
// workgroups g with g % 8 == i % 8, so the tiles that two ranks of one
// subdomain both read are shared through one L2.  Correctness does not depend
// on the placement: the exchange uses device-scope accesses.
__global__ void __launch_bounds__(SOLVE_THREADS) k_sweep(SweepArgs A) {
    constexpr int NW = SOLVE_THREADS / 64;
    constexpr int NWT = NW - 1;                    // tile waves
    constexpr int CW0 = NWT * 64;                  // first thread of the control wave
    constexpr int NRC = MAXR * TS / 64;            // own rows per control lane
    __shared__ double z[MAXMP];
    __shared__ double full[MAXMP];
    __shared__ double yw[NWT][MAXR * TS];
    __shared__ int sh_ok;

    const int mode = A.mode;
    int sub, rank;
    {
        const int x = blockIdx.x % 8, slot = blockIdx.x / 8;
        if (mode == 1) {
            if (x != 0) return;                        // idle slot
            sub = A.nsub;
            rank = slot;
        } else {
            const int P0 = A.subs[0].P;
            sub = x + 8 * (slot / P0);
            rank = slot % P0;
            if (sub >= A.nsub) return;                 // idle slot
        }
    }
    const SubDesc d = A.subs[sub];
    if (mode == 0 && A.done[d.pair]) return;   // uniform over the subdomain's ranks
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const bool ctl = wv == NWT;
    const int P = d.P, m = d.m, mp = d.mp, ms = d.ms, nt = d.nt, NT = d.NT;
    const int R = (NT - rank + P - 1) / P;         // block rows of this rank: rank + P*i, i < R
    const int ntw = R * NT;                        // tiles per phase for this rank
    const int nrow = R * TS;                       // rows finished by this rank
    const int64_t nn = (int64_t)A.W * A.H;
    const int64_t tstride = (int64_t)d.ntiles * TSZ;       // tiles of one line
    const double* __restrict__ Tb = A.factors + d.foff;
    const double* __restrict__ Bb = A.factors + d.boff;
    double* __restrict__ wst = A.work + d.woff;            // w_t, then x_t, of this rank's rows
    // published rows: [2][mp] pairs of 64-bit words (tag << 32 | half of the double)
    uint64_t* __restrict__ pub = reinterpret_cast<uint64_t*>(A.work + d.poff);
    DevStatus* st = A.status;
    const long long spin = A.spin_limit;
    const int nphase = 2 * nt - 1;
    const uint32_t epoch = A.epoch;

    // local unknown a of line t sits at global index gbase(a) + t * gstep
    const int64_t gstep = d.cols ? 1 : (int64_t)A.W;
    auto gbase = [&](int a) -> int64_t {
        const int s = a / 3, c = a % 3;
        const int x = d.cols ? d.bx0 : d.bx0 + s, y = d.cols ? d.by0 + s : d.by0;
        return ((int64_t)d.pair * 3 + c) * nn + (int64_t)y * A.W + x;
    };
    // right-hand side of row a = tid
    const double* __restrict__ rsrc = mode == 1 ? A.b_local + tid : A.r + (tid < m ? gbase(tid) : 0);
    const int64_t rstep = mode == 1 ? m : gstep;
    // B coefficient rows of this thread (forward: row a; backward: rows 3s.., 3s+3..)
    const int zs = tid / 3, ze = tid % 3;
    // this thread's tiles (fixed for all lines): offsets inside a line
    const int tj = lane & 31, th = lane >> 5;
    int64_t toff[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int qt = wv + NWT * p;
        const int I = rank + P * (qt / NT), J = qt % NT;
        const int k = J <= I ? I * (I + 1) / 2 + J : J * (J + 1) / 2 + I;
        toff[p] = (int64_t)k * TSZ + (16 * th) * TS + tj;
    }
    // own rows of the control lanes
    int crow[NRC];
#pragma unroll
    for (int i = 0; i < NRC; ++i) {
        const int k = tid - CW0 + 64 * i;
        crow[i] = k < nrow ? (rank + P * (k / TS)) * TS + k % TS : -1;
    }

    double pre[PF][16];
    double pr = 0.0, pb[6] = {0, 0, 0, 0, 0, 0};
    auto prefetch = [&](int q) {                    // tile waves
        const int t = q < nt ? q : 2 * nt - 2 - q;
        if (tid < m) {                              // z terms first: needed earlier
            if (q < nt) {
                pr = rsrc[t * rstep];
                if (t > 0) {
                    const double* cf = Bb + ((int64_t)t * m + tid) * 6;
#pragma unroll
                    for (int e = 0; e < 6; ++e) pb[e] = cf[e];
                }
            } else {
                const double* Bt = Bb + (int64_t)(t + 1) * m * 6;
#pragma unroll
                for (int c = 0; c < 3; ++c) pb[c] = Bt[(int64_t)(3 * zs + c) * 6 + 3 + ze];
#pragma unroll
                for (int c = 0; c < 3; ++c) pb[3 + c] = zs + 1 < ms ? Bt[(int64_t)(3 * (zs + 1) + c) * 6 + ze] : 0.0;
            }
        }
        const double* Tl = Tb + (int64_t)t * tstride;
#pragma unroll
        for (int p = 0; p < PF; ++p)
            if (wv + NWT * p < ntw) {
#pragma unroll
                for (int i = 0; i < 16; ++i) pre[p][i] = Tl[toff[p] + i * TS];
            }
    };
    double pw[NRC];
#pragma unroll
    for (int i = 0; i < NRC; ++i) pw[i] = 0.0;

    for (int i = tid; i < NWT * MAXR * TS; i += SOLVE_THREADS) (&yw[0][0])[i] = 0.0;
    if (!ctl) prefetch(0);
    // Phase structure (B = workgroup barrier):
    //   control wave: [gather(q)] B z B  .  B [finish, publish(q)]
    //   tile waves:              B z B [compute(q)] B [prefetch(q+1)]
    // Rows are exchanged as tagged 64-bit words (32-bit tag, 32-bit half of a
    // double): a reader polls the words it needs until both halves carry the
    // tag of the wanted phase, so one memory round trip both synchronises and
    // transfers the data; no separate flag, counter or store acknowledgement.
    __syncthreads();
    for (int q = 0; q < nphase; ++q) {
        const int t = q < nt ? q : 2 * nt - 2 - q;
        const bool fwd = q < nt;
        if (q > 0) {
            if (ctl) {
                // each lane needs mp/64 entries: issue all loads, then re-poll
                // only the entries whose tags are not there yet
                const uint32_t tag = epoch + (uint32_t)(q - 1);
                const uint64_t* pbuf = pub + (int64_t)((q - 1) & 1) * mp * 2;
                constexpr int NG = MAXMP / 64;
                uint64_t lo[NG], hi[NG];
                unsigned pending = 0;
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    if (lane + 64 * g < mp) pending |= 1u << g;
                long long n = 0;
                int ok = 1;
                while (pending) {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (pending & (1u << g)) {
                            const int a = lane + 64 * g;
                            lo[g] = __hip_atomic_load(const_cast<uint64_t*>(pbuf + 2 * a), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                            hi[g] = __hip_atomic_load(const_cast<uint64_t*>(pbuf + 2 * a + 1), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                        }
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if ((pending & (1u << g)) && (uint32_t)(lo[g] >> 32) == tag && (uint32_t)(hi[g] >> 32) == tag) {
                            full[lane + 64 * g] = __longlong_as_double((long long)((hi[g] << 32) | (lo[g] & 0xffffffffull)));
                            pending &= ~(1u << g);
                        }
                    if (!pending) break;
                    if (++n > spin ||
                        __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SF_ERR_DEVICE) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                // wave-wide outcome
                const int all_ok = __all(ok);
                if (lane == 0) {
                    if (!all_ok && atomicCAS(&st->code, 0, SF_ERR_DEVICE) == 0) {
                        st->sub = sub;
                        st->row = (int64_t)q;
                    }
                    sh_ok = all_ok;
                }
            }
            __syncthreads();
            if (!sh_ok) return;
        }
        // z: forward r_t - B_t w_{t-1}; backward B_{t+1}^T x_{t+1}
        if (!ctl && tid < mp) {
            double v = 0.0;
            if (tid < m) {
                if (fwd) {
                    v = pr;
                    if (t > 0) {
                        double bw = 0.0;
                        if (zs > 0)
#pragma unroll
                            for (int e = 0; e < 3; ++e) bw = fma(pb[e], full[3 * (zs - 1) + e], bw);
#pragma unroll
                        for (int e = 0; e < 3; ++e) bw = fma(pb[3 + e], full[3 * zs + e], bw);
                        v -= bw;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < 3; ++c) v = fma(pb[c], full[3 * zs + c], v);
                    if (zs + 1 < ms)
#pragma unroll
                        for (int c = 0; c < 3; ++c) v = fma(pb[3 + c], full[3 * (zs + 1) + c], v);
                }
            }
            z[tid] = v;
        }
        __syncthreads();
        if (!ctl) {
            // this rank's block rows
#pragma unroll
            for (int p = 0; p < PF; ++p) {
                const int qt = wv + NWT * p;
                if (qt < ntw) {
                    const int i = qt / NT;
                    tile_apply(pre[p], rank + P * i, qt % NT, z, &yw[wv][i * TS]);
                }
            }
            for (int qt = wv + NWT * PF; qt < ntw; qt += NWT) {
                const int i = qt / NT;
                double tv[16];
                load_tile(Tb + (int64_t)t * tstride, rank + P * i, qt % NT, tv);
                tile_apply(tv, rank + P * i, qt % NT, z, &yw[wv][i * TS]);
            }
        }
        __syncthreads();
        if (!ctl) {
            if (q + 1 < nphase) prefetch(q + 1);
        } else {
            // finish and publish this rank's rows; keep them; prefetch w
            const uint64_t tag = (uint64_t)(epoch + (uint32_t)q) << 32;
            uint64_t* pout = pub + (int64_t)(q & 1) * mp * 2;
            double* wt = wst + (int64_t)t * mp;
#pragma unroll
            for (int i = 0; i < NRC; ++i) {
                const int k = tid - CW0 + 64 * i;
                if (crow[i] >= 0) {
                    double y = 0.0;
                    for (int w = 0; w < NWT; ++w) {
                        y += yw[w][k];
                        yw[w][k] = 0.0;
                    }
                    if (!fwd) y = pw[i] - y;               // x_t = w_t - S_t^{-1} v
                    const uint64_t bits = (uint64_t)__double_as_longlong(y);
                    __hip_atomic_store(pout + 2 * crow[i], tag | (bits & 0xffffffffull), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_store(pout + 2 * crow[i] + 1, tag | (bits >> 32), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    wt[crow[i]] = y;                               // w_t or x_t
                }
            }
            if (q + 1 < nphase && q + 1 >= nt) {
                const double* wn = wst + (int64_t)(2 * nt - 3 - q) * mp;   // line of phase q + 1
#pragma unroll
                for (int i = 0; i < NRC; ++i) pw[i] = crow[i] >= 0 ? wn[crow[i]] : 0.0;
            }
        }
    }
    // U[O_i] += x on the owned nodes of this rank's rows (x_{nt-1} = w_{nt-1})
    __syncthreads();
    for (int i = tid; i < nt * nrow; i += SOLVE_THREADS) {
        const int t = i / nrow, k = i % nrow;
        const int a = (rank + P * (k / TS)) * TS + k % TS;
        if (a >= m) continue;
        const double v = wst[(int64_t)t * mp + a];
        if (mode == 1) {
            A.x_local[(int64_t)t * m + a] = v;
            continue;
        }
        int x, y;
        local_to_global(d, t, a / 3, x, y);
        if (x >= d.ox0 && x < d.ox1 && y >= d.oy0 && y < d.oy1)
            A.U[((int64_t)d.pair * 3 + a % 3) * nn + (int64_t)y * A.W + x] += v;
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
    a.nsub = single_sub >= 0 ? single_sub : c->nsub;
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
    // tags must differ from every tag left in the exchange buffers by earlier
    // launches: advance by more than the phases of one launch
    a.epoch = c->sweep_epoch;
    int maxph = 0;
    for (const auto& d : c->subs) maxph = std::max(maxph, 2 * d.nt);
    c->sweep_epoch += (uint32_t)maxph + 2;
    const int grid = single_sub >= 0 ? 8 * c->maxP : c->sweep_grid;
    const void* kern = (const void*)k_sweep;
    void* args[] = {&a};
    if (c->maxP > 1) {
        if (hipLaunchCooperativeKernel(kern, dim3(grid), dim3(SOLVE_THREADS), args, 0, c->stream) != hipSuccess)
            return SF_ERR_HIP;
    } else {
        if (hipLaunchKernel(kern, dim3(grid), dim3(SOLVE_THREADS), args, 0, c->stream) != hipSuccess)
            return SF_ERR_HIP;
    }
    return SF_OK;
}

}  // namespace sfdd

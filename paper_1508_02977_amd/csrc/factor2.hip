// Subdomain factorisation, cooperative form: Pf workgroups per subdomain.
//
// Same factor as factor.hip (paper, Section 3.2, local direct solves): for
// every line t of a subdomain, S_t = A_tt - B_t S_{t-1}^{-1} B_t^T and its
// inverse, stored as 32x32 lower tiles.  Here the inverse is formed by the
// blocked symmetric sweep (Gauss-Jordan without pivoting, valid because S_t
// is SPD): for each 32-column pivot block k,
//     Pi = S_kk^{-1}
//     S_ij <- S_ij - S_ik Pi S_kj        (i, j != k)
//     S_ik <- S_ik Pi,  S_kj <- Pi S_kj,  S_kk <- -Pi
// and after all NT pivots the matrix holds -S^{-1}.  The pivot blocks are the
// Schur complements a Cholesky factorisation would meet, so a non-positive
// pivot inside Pi flags SF_NOT_SPD exactly as before.
//
// Work split: rank r owns block rows r and NT-1-r (balanced: NT+1 lower tiles
// per rank) and keeps its tiles in MFMA accumulators (v_mfma_f64_16x16x4f64,
// one 16x16 block per accumulator) for the whole line.  Lane layout of that
// instruction (checked on gfx950): A[i][k] in lane i + 16k, B[k][j] in lane
// j + 16k, accumulator element q of lane l is D[l/16 + 4q][l%16].
//
// Each pivot step needs block column k of the current matrix: its owners
// publish it to a global exchange slot (relaxed device-scope stores) and bump
// the chain's counter, and every rank reads it into LDS.  One more workgroup
// per chain, the pivot server, forms every Pi: the owner of block row k+1
// updates its diagonal tile first in pivot step k and hands it over, so
// Pi_{k+1} is ready by the time the ranks finish the rest of step k.  Pivot
// blocks and Pi travel as tagged 64-bit words (32-bit tag, half of a double),
// so one poll both synchronises and transfers them.  The Schur update of the
// next line is built from the full symmetric S_{t-1}^{-1} that the ranks leave
// in global memory at the end of a line.
#include <algorithm>
#include <cmath>

#include "element.h"
#include "factor2_layout.h"
#include "sfdd_internal.h"

namespace sfdd {

constexpr int F2_THREADS = 256;      // one wave per SIMD: 512 registers per wave
constexpr int F2_NW = F2_THREADS / 64;
constexpr int F2_MAXNT = 24;          // line matrices up to 768 x 768
constexpr int LDP = 34;               // LDS row pitch (doubles): conflict-free 16x4 / 4x16 fragments
constexpr int LTILE = TS * LDP;       // doubles per LDS tile
// LDS tiles of the exchange column a rank keeps: every block column when one
// rank owns a row pair (NT <= 12); with split pairs the columns of the rank's
// parity (at most 12) and its two rows (slots 12, 13)
constexpr int F2_SLOTS = 14;
constexpr int F2_XSLOT_A = 12, F2_XSLOT_B = 13;

// The ranks keep the exchange column in LDS as 32x32 tiles of pitch 32 with
// the 16-byte chunks of row r permuted by r mod 16 (chunk ch at position
// ch ^ (r & 15)): a 64-lane load then lands 1 KB contiguously (direct
// global-to-LDS loads), and the 16x4 operand fragments of the MFMA reads
// fall on distinct banks.
__device__ __forceinline__ int colk_at(int slot, int r, int c) {
    return slot * TSZ + r * TS + ((((c >> 1) ^ (r & 15))) << 1) + (c & 1);
}
constexpr int F2_MAXBLK = 13;         // accumulator blocks per wave: 4 * 13 tiles / 4 waves
static_assert(F2_NW == F2_WAVES && F2_MAXBLK == F2_BLOCKS, "factor workspace layout");
static_assert(F2_NW * 12 * 256 <= F2_SLOTS * TSZ, "final-write staging fits the exchange column's LDS");
static_assert(2 * F2_SPLIT_NT == F2_MAXNT && F2_XSLOT_B < F2_SLOTS, "split ranks: parity slots, then the two rows");

// The tiles a rank owns: block rows rowA = rp and rowB = NT-1-rp (one row if
// they coincide), and in them every block column J <= the row (sp = 1) or the
// columns J = h (mod 2) (sp = 2, half h of the pair).  Tile q of the rank's
// list: the row-A tiles by increasing J, then the row-B tiles.
struct F2Own {
    int rowA, rowB, nrows, h, sp, ntA, ntl;
};
__device__ __forceinline__ F2Own f2_own(int rank, int NT) {
    F2Own o;
    o.sp = f2_split(NT);
    o.h = rank % o.sp;
    o.rowA = rank / o.sp;
    o.rowB = NT - 1 - o.rowA;
    o.nrows = o.rowB > o.rowA ? 2 : 1;
    o.ntA = o.rowA >= o.h ? (o.rowA - o.h) / o.sp + 1 : 0;
    const int ntB = o.nrows == 2 && o.rowB >= o.h ? (o.rowB - o.h) / o.sp + 1 : 0;
    o.ntl = o.ntA + ntB;
    return o;
}
// LDS slot of block column J of the exchange column (J a column the rank
// reads: one of its tile columns or one of its rows)
__device__ __forceinline__ int f2_slot(const F2Own& o, int J) {
    if (o.sp == 1) return J;
    if ((J & 1) == o.h) return J >> 1;
    return J == o.rowA ? F2_XSLOT_A : F2_XSLOT_B;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));

// Arithmetic of the ranks' tiles: FP64 (v_mfma_f64_16x16x4f64) or FP32
// (v_mfma_f32_16x16x4f32).  Both take A[i][k] in lane i + 16k and B[k][j] in
// lane j + 16k; they differ in where an accumulator element lives (checked
// on gfx950): FP64 element q of lane l is D[l/16 + 4q][l%16], FP32 element q
// is D[4(l/16) + q][l%16].  LDS tiles of the exchange column keep rows of 32
// values with the 16-byte chunks of row r permuted (chunk c at c ^ (r mod the
// chunks per row)); the pivot and X tiles use a row pitch that keeps 16-byte
// reads aligned.
template <typename T> struct F2T;
template <> struct F2T<double> {
    using V4 = d4;
    static constexpr int LDPT = 34;       // LDS row pitch of the pivot / X tiles
    static constexpr int EPC = 2;         // values per 16-byte chunk
    __device__ static __forceinline__ V4 mfma(double a, double b, V4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int cr, int q) { return cr + 4 * q; }
};
template <> struct F2T<float> {
    using V4 = f4;
    static constexpr int LDPT = 36;
    static constexpr int EPC = 4;
    __device__ static __forceinline__ V4 mfma(float a, float b, V4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int cr, int q) { return 4 * cr + q; }
};
template <typename T>
__device__ __forceinline__ int colk_at_t(int slot, int r, int c) {
    constexpr int E = F2T<T>::EPC, CPR = TS / E;   // chunks per row
    return slot * TSZ + r * TS + (((c / E) ^ (r & (CPR - 1))) * E) + (c & (E - 1));
}

struct FactorArgs {
    const SubDesc* subs;
    int sub0, nsub;           // subdomains [sub0, nsub) of this launch
    int lanes;                // subdomains side by side in the grid (8: one XCD each)
    int nmain;                // the first nmain of them side by side; each later one takes
                              // the next groups x (pf + 1) workgroups (ranks spread over XCDs)
    int pf;                   // rank slots per chain (the largest f2_ranks(NT))
    int groups;               // chains per subdomain: 1 (top to bottom) or 2 (twisted)
    int fp32;                 // 1: store the inverse tiles in single precision
    const double* f0;
    const double* al;
    double* factors;
    double* work;
    uint32_t* counters;
    DevStatus* status;
    int W, H;
    double lam;
    long long spin_limit;
    uint32_t epoch;           // tag base of this launch (pivot-block and Pi words carry epoch + pivot)
    double ptol;              // a pivot p is accepted when p > ptol x the diagonal entry of A_tt it came from
    int32_t* fail;            // [subdomains] set to 1 where a pivot is rejected (or null)
    const int32_t* sublist;   // if set: the launch factors subdomains sublist[0 .. nsub - sub0)
};

// Line coefficients of every subdomain, computed once before the
// factorisation: per line t and node s the 3x3 blocks A[(t,s),(t,s)] and
// A[(t,s),(t,s+1)] (row-major, 18 doubles at aoff + (t*ms + s)*18) and the
// coupling rows B_t[3s+c][.] (6 doubles per row, boff + (t*m + 3s+c)*6).
__global__ void k_line_coeffs(const SubDesc* __restrict__ subs, const double* __restrict__ f0_all,
                              const double* __restrict__ al_all, double* __restrict__ factors, int W, int H,
                              double lam, int sub0, const double* __restrict__ coef_all) {
    const SubDesc d = subs[sub0 + blockIdx.y];
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)d.nt * d.ms) return;
    const int t = (int)(idx / d.ms), s = (int)(idx % d.ms);
    const int64_t nn = (int64_t)W * H, ne = (int64_t)(W - 1) * (H - 1) * 2;
    const double* f0 = f0_all + d.pair * nn;
    const double* al = al_all + d.pair * ne;
    const double* cf = coef_all ? coef_all + (int64_t)d.pair * CLG_NCOEF * ne : nullptr;   // K_rho data term
    double* Ab = factors + d.aoff + idx * 18;
    int x, y;
    local_to_global(d, t, s, x, y);
    double blk[9];
    stencil_block(f0, al, W, H, x, y, 0, 0, lam, blk, cf);
    for (int k = 0; k < 9; ++k) Ab[k] = blk[k];
    if (s + 1 < d.ms) {
        if (d.cols) stencil_block(f0, al, W, H, x, y, 0, 1, lam, blk, cf);
        else        stencil_block(f0, al, W, H, x, y, 1, 0, lam, blk, cf);
    } else {
        for (int k = 0; k < 9; ++k) blk[k] = 0.0;
    }
    for (int k = 0; k < 9; ++k) Ab[9 + k] = blk[k];
    if (t > 0) {
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
        double* row = factors + d.boff + ((int64_t)t * d.m + 3 * s) * 6;
        for (int c = 0; c < 3; ++c)
            for (int e = 0; e < 3; ++e) {
                row[c * 6 + e] = bd[3 * e + c];        // B[3s+c][3(s-1)+e]
                row[c * 6 + 3 + e] = bs[3 * e + c];    // B[3s+c][3s+e]
            }
    }
}

// One 16-byte global-to-LDS load per lane, device-scope coherent (sc1).  Kept
// out of the kernel template: its LDS address-space cast has no meaning in the
// host compilation, which instantiates the template to emit its launch stub.
__device__ __forceinline__ void f2_load_lds16(const void* src, void* lds) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 16 /* sc1 */);
}

template <typename T>
__device__ __forceinline__ void xstore(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T xload(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool f2_wait(uint32_t* cnt, uint32_t target, const FactorArgs& A, int sub, int* sh_ok) {
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

__device__ __forceinline__ void f2_signal(uint32_t* cnt) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A value as tagged 64-bit words (32-bit tag, 32 bits of the value): a
// double takes two words, a float one; entry i of a tile sits at word
// 2 i either way.
__device__ __forceinline__ void f2_tstore(uint64_t* p, uint32_t tag, double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v), tg = (uint64_t)tag << 32;
    __hip_atomic_store(p, tg | (bits & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(p + 1, tg | (bits >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void f2_tstore(uint64_t* p, uint32_t tag, float v) {
    const uint64_t bits = (uint64_t)__float_as_uint(v), tg = (uint64_t)tag << 32;
    __hip_atomic_store(p, tg | bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll the 32x32 tile of tagged words (values of type TW) at src until every
// entry carries `tag`; entry i = tix + 256 u (tix: this thread's index) goes
// to the LDS tile dst (pitch ldp, type TD) as soon as it is seen.  False (and
// SF_ERR_DEVICE) when the wait is abandoned; the result is uniform over the
// workgroup.
template <typename TW, typename TD>
__device__ __forceinline__ bool f2_tpoll(const uint64_t* src, uint32_t tag, TD* dst, int ldp, const DevStatus* stc, DevStatus* st,
                         long long spin, int sub, int tix) {
    constexpr int NU = TSZ / 256;
    constexpr bool W2 = sizeof(TW) == 8;
    unsigned pending = (1u << NU) - 1;
    long long n = 0;
    int ok = 1;
    while (pending) {
        uint64_t lo[NU], hi[NU];
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if (pending & (1u << u)) {
                const uint64_t* w = src + 2 * (tix + 256 * u);
                lo[u] = __hip_atomic_load(const_cast<uint64_t*>(w), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                hi[u] = W2 ? __hip_atomic_load(const_cast<uint64_t*>(w + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : lo[u];
            }
#pragma unroll
        for (int u = 0; u < NU; ++u)
            if ((pending & (1u << u)) && (uint32_t)(lo[u] >> 32) == tag && (uint32_t)(hi[u] >> 32) == tag) {
                const int i = tix + 256 * u;
                TD v;
                if constexpr (W2) v = (TD)__longlong_as_double((long long)((hi[u] << 32) | (lo[u] & 0xffffffffull)));
                else v = (TD)__uint_as_float((unsigned)(lo[u] & 0xffffffffull));
                dst[(i / TS) * ldp + i % TS] = v;
                pending &= ~(1u << u);
            }
        if (!pending) break;
        if (++n > spin || __hip_atomic_load(&stc->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SF_ERR_DEVICE) {
            ok = 0;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    if (!ok && atomicCAS(&st->code, 0, SF_ERR_DEVICE) == 0) {
        st->sub = sub;
        st->row = (int64_t)tag;
    }
    return __syncthreads_and(ok) != 0;
}

__device__ __forceinline__ void f2_tile_of(int q, const F2Own& o, int& I, int& J) {
    if (q < o.ntA) { I = o.rowA; J = o.h + o.sp * q; }
    else           { I = o.rowB; J = o.h + o.sp * (q - o.ntA); }
}

// Publish block column `col` of the current matrix (the own blocks in it)
// into the exchange slots xb[J] = S_{J,col} (32x32 row-major).
template <typename T>
__device__ __forceinline__ void f2_publish(const typename F2T<T>::V4 (&acc)[F2_MAXBLK], T* xb, int col, int nblk,
                                           const F2Own& o, int wv, int cr, int cc) {
#pragma unroll
    for (int b = 0; b < F2_MAXBLK; ++b) {
        const int blk = wv + F2_NW * b;
        if (blk >= nblk) continue;
        int I, J;
        f2_tile_of(blk >> 2, o, I, J);
        const int qi = (blk >> 1) & 1, qj = blk & 1;
        if (J == col) {                                  // tile (I, col): slot I as is
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xstore(xb + (int64_t)I * TSZ + (16 * qi + F2T<T>::row(cr, q)) * TS + 16 * qj + cc, acc[b][q]);
        } else if (I == col) {                           // tile (col, J), J < col: slot J transposed
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xstore(xb + (int64_t)J * TSZ + (16 * qj + cc) * TS + 16 * qi + F2T<T>::row(cr, q), acc[b][q]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Pi = S_kk^{-1} of the symmetric 32x32 tile Sk (LDS, pitch LDP) into piv, by
// one wave, with 2x2 blocks of 16.  With S_kk = [[A, B^T], [B, C]]
// (symmetrised on load): A^-1 and C'^-1, C' = C - B A^-1 B^T, by the symmetric
// sweep (16 steps each, every lane holding 4 entries in the MFMA accumulator
// layout); then with X = B A^-1 on FP64 MFMA:
// Pi = [[A^-1 + X^T C'^-1 X, -(C'^-1 X)^T], [-C'^-1 X, C'^-1]].
// The pivots met are those of the unblocked sweep; each is checked against
// the diagonal entry of A_tt it came from (adiag_k, LDS).
// Publish the own diagonal tile (col, col) as tagged words into the pivot-block slot db.
template <typename T>
__device__ __forceinline__ void f2_publish_diag(const typename F2T<T>::V4 (&acc)[F2_MAXBLK], uint64_t* db, uint32_t tag,
                                                int col, int nblk, const F2Own& o, int wv, int cr, int cc) {
#pragma unroll
    for (int b = 0; b < F2_MAXBLK; ++b) {
        const int blk = wv + F2_NW * b;
        if (blk >= nblk) continue;
        int I, J;
        f2_tile_of(blk >> 2, o, I, J);
        const int qi = (blk >> 1) & 1, qj = blk & 1;
        if (I == col && J == col) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                f2_tstore(db + 2 * ((16 * qi + F2T<T>::row(cr, q)) * TS + 16 * qj + cc), tag, (T)acc[b][q]);
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// Cross-lane moves of the pivot sweep, all in the VALU.  A 16x16 block sits
// in a wave as element q of lane (ci, ri) = row ri + 4q, column ci
// (lane = ci + 16 ri).  Broadcast of lane row R (lanes 16R..16R+15) to all
// four: permlane16_swap(x, x) yields rows (0,0,2,2) and (1,1,3,3),
// permlane32_swap(x, x) the lower and the upper half twice (checked on
// gfx950).
template <int R>
__device__ __forceinline__ double f2_bcast_row(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    const auto l1 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h1 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    lo = (R & 1) ? l1[1] : l1[0];
    hi = (R & 1) ? h1[1] : h1[0];
    const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    lo = (R & 2) ? l2[1] : l2[0];
    hi = (R & 2) ? h2[1] : h2[0];
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// lane L of every 16-lane row to the whole row (DPP row_newbcast)
template <int L>
__device__ __forceinline__ double f2_row_lane(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0x150 + L, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x150 + L, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double f2_lane(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// Gauss-Jordan step on pivot P of the 16x16 block v (see f2_pivot_inverse):
// row P from its lane row, column P from lane P of every row, the pivot by
// readlane.  The pivot test is recorded in bad (first failing pivot).
template <int P>
__device__ __forceinline__ void f2_gj_step(double (&v)[4], const double (&adg)[16], int ci, int ri, int& bad) {
    constexpr int Q = P >> 2, R = P & 3;
    const double rowp = f2_bcast_row<R>(v[Q]);               // M[P][ci]
    double colp[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) colp[q] = f2_row_lane<P>(v[q]);   // M[ri + 4q][P]
    const double pp = f2_lane(v[Q], P + 16 * R);             // M[P][P]
    const bool okp = pp > adg[P] && isfinite(pp);      // adg: the pivot threshold
    bad = (bad < 0 && !okp) ? P : bad;
    double ip = __builtin_amdgcn_rcp(pp);
    ip = fma(fma(-pp, ip, 1.0), ip, ip);
    ip = fma(fma(-pp, ip, 1.0), ip, ip);
    const bool jp = ci == P;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool iq = ri + 4 * q == P;
        const double upd = v[q] - colp[q] * rowp * ip;
        const double side = jp ? colp[q] * ip : upd;
        v[q] = iq ? (jp ? -ip : rowp * ip) : side;
    }
}
template <int P>
struct F2Sweep {
    __device__ static __forceinline__ void run(double (&v)[4], const double (&adg)[16], int ci, int ri, int& bad) {
        f2_gj_step<P>(v, adg, ci, ri, bad);
        F2Sweep<P + 1>::run(v, adg, ci, ri, bad);
    }
};
template <>
struct F2Sweep<16> {
    __device__ static __forceinline__ void run(double (&)[4], const double (&)[16], int, int, int&) {}
};

__device__ __forceinline__ void f2_pivot_inverse(const double* Sk, double* piv, double* xr, const double* adiag_k, int lane,
                                 DevStatus* status, int sub, int64_t row0, double ptol, int32_t* fail) {
    constexpr int PB = 17;                        // pitch of the 16x16 scratch blocks
    double* bA = xr;                              // A^-1
    double* bB = bA + 16 * PB;                    // B, then -C'^-1 X
    double* bX = bB + 16 * PB;                    // X = B A^-1
    double* bC = bX + 16 * PB;                    // C'^-1
    const int ci = lane & 15, ri = lane >> 4;     // element q of a lane: row ri + 4q, column ci
    d4 Av, Bv, Cv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = ri + 4 * q, j = ci;
        Av[q] = 0.5 * (Sk[i * LDP + j] + Sk[j * LDP + i]);
        Bv[q] = 0.5 * (Sk[(16 + i) * LDP + j] + Sk[j * LDP + 16 + i]);
        Cv[q] = 0.5 * (Sk[(16 + i) * LDP + 16 + j] + Sk[(16 + j) * LDP + 16 + i]);
    }
    // v (16x16) <- -v^{-1} by Gauss-Jordan without pivoting.  The pivot test
    // is recorded per step and reported once after the sweep (first failing
    // pivot), and 1/pp is the hardware reciprocal refined by two Newton steps
    // r <- r + r (1 - pp r), which keeps every step of this latency-bound chain
    // short; rows, columns and the pivot move between lanes without LDS.
    auto sweep16 = [&](d4& v, int poff) {
        double adg[16];
#pragma unroll
        for (int p = 0; p < 16; ++p) adg[p] = ptol * adiag_k[poff + p];
        double w[4] = {v[0], v[1], v[2], v[3]};
        int bad = -1;
        F2Sweep<0>::run(w, adg, ci, ri, bad);
#pragma unroll
        for (int q = 0; q < 4; ++q) v[q] = w[q];
        if (lane == 0 && bad >= 0) {
            if (fail) fail[sub] = 1;
            if (atomicCAS(&status->code, 0, SF_NOT_SPD) == 0) {
                status->sub = sub;
                status->row = row0 + poff + bad;
            }
        }
    };
    auto put = [&](double* buf, const d4& v, double sgn) {
#pragma unroll
        for (int q = 0; q < 4; ++q) buf[(ri + 4 * q) * PB + ci] = sgn * v[q];
    };
    // D = op(P) op(Q) on MFMA; operand rows from 16x16 scratch blocks
    auto mm = [&](const double* P, bool Pt, const double* Q, bool Qt) -> d4 {
        const int ii = lane & 15, kk = lane >> 4;
        d4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kx = 4 * ks + kk;
            const double a = Pt ? P[kx * PB + ii] : P[ii * PB + kx];
            const double b = Qt ? Q[ii * PB + kx] : Q[kx * PB + ii];
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
        }
        return d;
    };
    auto sync_lds = [&]() {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    sweep16(Av, 0);                               // Av = -A^-1
    put(bA, Av, -1.0);
    put(bB, Bv, 1.0);
    sync_lds();
    const d4 Xv = mm(bB, false, bA, false);       // X = B A^-1
    put(bX, Xv, 1.0);
    sync_lds();
    const d4 T = mm(bX, false, bB, true);         // X B^T
    d4 Cp;
#pragma unroll
    for (int q = 0; q < 4; ++q) Cp[q] = Cv[q] - T[q];
    sweep16(Cp, 16);                              // Cp = -C'^-1
    put(bC, Cp, -1.0);
    sync_lds();
    d4 P21 = mm(bC, false, bX, false);            // C'^-1 X
#pragma unroll
    for (int q = 0; q < 4; ++q) P21[q] = -P21[q];
    put(bB, P21, 1.0);
    sync_lds();
    const d4 T3 = mm(bX, true, bB, false);        // X^T (-C'^-1 X)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int i = ri + 4 * q, j = ci;
        piv[i * LDP + j] = -Av[q] - T3[q];                  // A^-1 + X^T C'^-1 X
        piv[(16 + i) * LDP + j] = P21[q];                   // -C'^-1 X
        piv[j * LDP + 16 + i] = P21[q];                     // its transpose
        piv[(16 + i) * LDP + 16 + j] = -Cp[q];              // C'^-1
    }
}

template <typename T>
__global__ void __launch_bounds__(F2_THREADS) k_factor2(FactorArgs A) {
    using V4 = typename F2T<T>::V4;
    constexpr int LDPT = F2T<T>::LDPT, LTT = TS * LDPT;
    // LDS: exchange column (the rank's F2_SLOTS tiles), then pivot inverse and
    // scaled rows X_I (2 tiles).  While a line is built, the exchange column's
    // space holds the line's node blocks and couplings, and the pivot / X
    // space the waves' window scratch.
    __shared__ __attribute__((aligned(16))) T colk[F2_SLOTS * TSZ];
    __shared__ __attribute__((aligned(16))) T pxr[3 * LTT];
    T* const piv = pxr;
    T* const xr = pxr + LTT;
    __shared__ int sh_ok;

    // workgroup g runs on XCD g % 8: with A.lanes = 8 the ranks of subdomain
    // i < nmain are the slots with g % 8 == i % 8, so its exchange stays
    // inside one L2; a subdomain i >= nmain (filling the workgroups that the
    // side-by-side groups leave) has per contiguous workgroups.  Per chain:
    // ranks 0..pf-1 and the pivot server (rank pf)
    const int ps = A.pf + 1, per = A.groups * ps;
    const int mainwg = A.lanes * ((A.nmain + A.lanes - 1) / A.lanes) * per;
    int local, within;
    if ((int)blockIdx.x < mainwg) {
        const int slot = blockIdx.x / A.lanes;
        local = (int)(blockIdx.x % A.lanes) + A.lanes * (slot / per);
        within = slot % per;
        if (local >= A.nmain) return;                    // idle slot
    } else {
        const int b = (int)blockIdx.x - mainwg;
        local = A.nmain + b / per;
        within = b % per;
    }
    const int chain = within / ps, rank = within % ps;
    const bool server = rank == A.pf;
    if (local >= A.nsub - A.sub0) return;                // idle slot
    const int sub = A.sublist ? A.sublist[local] : A.sub0 + local;
    const SubDesc d = A.subs[sub];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int m = d.m, mp = d.mp, NT = d.NT, ms = d.ms;
    const int Pf = f2_ranks(NT);
    if (!server && rank >= Pf) return;                   // surplus slot of a short subdomain
    double* Tout = A.factors + d.foff;
    double* Bst = A.factors + d.boff;
    // per chain: the full symmetric inverse of its latest line (mp x mp),
    // [2][NT][32x32] exchange slots, then per rank and wave F2_MAXBLK 16x16
    // blocks of build scratch
    const int64_t cstride = f2_chain_doubles(mp, NT);   // (in doubles; values of type T from its start)
    T* Sup = reinterpret_cast<T*>(A.work + d.soff);                   // top chain: S_{t-1}^{-1}
    T* Sdn = reinterpret_cast<T*>(A.work + d.soff + cstride);         // bottom chain: S_{t+1}^{-1}
    T* Sown = chain == 0 ? Sup : Sdn;
    T* xch = Sown + (int64_t)mp * mp;
    uint64_t* dslot = reinterpret_cast<uint64_t*>(xch + 2ll * NT * TSZ);   // [2][TSZ] tagged pivot blocks
    uint64_t* pslot = dslot + 4 * TSZ;                                        // [2][TSZ] tagged Pi
    T* bscr = reinterpret_cast<T*>(pslot + 4 * TSZ) + (int64_t)(rank * F2_NW + wv) * F2_MAXBLK * 256;
    uint32_t* cnt = A.counters + F2_COUNTERS * (2 * sub + chain);   // column parts published

    const int nt = d.nt, km = d.kmid;
    const int nl1 = nt - 1 - km;                       // lines of the bottom chain
    const int nlines = chain == 0 ? km + 1 : nl1;
    if (server) {
        // pivot server: for every pivot of every line of the chain, wait for
        // the pivot block S_kk, form Pi_k (wave 0) and publish it
        // FP64 scratch in the exchange column's LDS: pivot block, Pi, the
        // pivot inverse's 16x16 blocks, the diagonal of A_tt
        uint32_t npiv = 0;
        double* const sd = reinterpret_cast<double*>(colk);
        double* const sk = sd;                   // 32 x LDP
        double* const spiv = sd + LTILE;         // 32 x LDP
        double* const sxr = sd + 2 * LTILE;      // 4 blocks of 16 x 17
        double* const adiag = sd + 3 * LTILE;    // mp
        static_assert(3 * LTILE + F2_MAXNT * TS <= F2_SLOTS * TSZ / 2, "server scratch fits the exchange column");
        for (int li = 0; li < nlines; ++li) {
            const int t = chain == 0 ? li : nt - 1 - li;
            const double* Ag = A.factors + d.aoff + (int64_t)t * ms * 18;
            for (int a = tid; a < mp; a += F2_THREADS) adiag[a] = a < m ? Ag[18 * (a / 3) + 4 * (a % 3)] : 1.0;
            for (int k = 0; k < NT; ++k) {
                ++npiv;
                if (!f2_tpoll<T, double>(dslot + (npiv & 1) * 2 * TSZ, A.epoch + npiv, sk, LDP, A.status, A.status,
                                         A.spin_limit, sub, tid))
                    return;
                if (wv == 0)
                    f2_pivot_inverse(sk, spiv, sxr, adiag + k * TS, lane, A.status, sub, (int64_t)t * m + k * TS, A.ptol,
                                     A.fail);
                __syncthreads();
                uint64_t* pb = pslot + (npiv & 1) * 2 * TSZ;
                for (int i = tid; i < TSZ; i += F2_THREADS)
                    f2_tstore(pb + 2 * i, A.epoch + npiv, (T)spiv[(i / TS) * LDP + i % TS]);
            }
        }
        return;
    }

    // own block rows and tiles; tile list: row rowA first, then row rowB
    const F2Own own = f2_own(rank, NT);
    const int rowA = own.rowA, rowB = own.rowB, nrows = own.nrows;
    const int nblk = 4 * own.ntl;             // 16x16 accumulator blocks
    // exchange-column tiles this rank reads, in load order: every block column
    // (sp = 1), or the npar columns of its parity and then its rows of the
    // other parity (sp = 2); f2_slot gives each one's LDS slot
    const int npar = own.sp == 1 ? NT : (NT - own.h + 1) / 2;
    const bool xtraA = own.sp == 2 && (rowA & 1) != own.h;
    const bool xtraB = own.sp == 2 && nrows == 2 && (rowB & 1) != own.h;
    const int nslots = npar + (xtraA ? 1 : 0) + (xtraB ? 1 : 0);
    V4 acc[F2_MAXBLK];
    // fragment coordinates of this lane inside a 16x16 block
    // (recomputed from an opaque copy of the lane id in every pivot step, so
    // that the compiler does not keep the dozens of loop-invariant LDS
    // addresses of the unrolled block loops live across the whole line)
    int fr = lane & 15, fk = lane >> 4;                    // A/B operand: row fr, k-slice fk
    int cr = lane >> 4, cc = lane & 15;                    // accumulator element q: row F2T<T>::row(cr, q), col cc

    // Lines of the chains: the top chain (0) takes lines 0..k-1 and then the
    // middle line k, the bottom chain (1) lines nt-1..k+1 (k = d.kmid; with one
    // chain k = nt - 1).  Top line t: S_t = A_tt - B_t S_{t-1}^{-1} B_t^T.
    // Bottom line t: S_t = A_tt - B_{t+1}^T S_{t+1}^{-1} B_{t+1}.  Middle: both
    // terms, after the bottom chain has finished.
    uint32_t phase = 0, npiv = 0;
    for (int li = 0; li < nlines; ++li) {
        const int t = chain == 0 ? li : nt - 1 - li;
        const bool mid = chain == 0 && li == km;
        const bool hup = chain == 0 && t > 0;                    // term of line t-1
        const bool hdn = (chain == 1 || mid) && t < nt - 1;      // term of line t+1
        // ---------- phase 0 of the line: build own tiles of S_t -------------
        // A_tt node blocks and the couplings of this line into LDS
        T* Aself = colk;                         // [ms][9]
        T* Anext = colk + 9 * ms;                // [ms][9]: block (s, s+1)
        T* Bl = colk + 18 * ms;                  // [m][6]: B_t, nodes s-1, s of line t-1
        T* Cl = Bl + 6 * m;                      // [m][6]: B_{t+1}^T, nodes s, s+1 of line t+1
        {
            const double* Ag = A.factors + d.aoff + (int64_t)t * ms * 18;
            for (int i = tid; i < 18 * ms; i += F2_THREADS) {
                const int s = i / 18, k = i % 18;
                if (k < 9) Aself[9 * s + k] = Ag[i];
                else       Anext[9 * s + k - 9] = Ag[i];
            }
            if (hup) {
                const double* Bg = Bst + (int64_t)t * m * 6;
                for (int i = tid; i < 6 * m; i += F2_THREADS) Bl[i] = Bg[i];
            }
            if (hdn) {
                // B_{t+1}^T as rows of line t: node s couples to nodes s, s+1 of line t+1
                const double* Bg = Bst + (int64_t)(t + 1) * m * 6;
                for (int i = tid; i < 6 * m; i += F2_THREADS) {
                    const int a = i / 6, k = i % 6, s = a / 3, c = a % 3, g = k % 3;
                    double v = 0.0;
                    if (k < 3) v = Bg[(3 * s + g) * 6 + 3 + c];
                    else if (s + 1 < ms) v = Bg[(3 * (s + 1) + g) * 6 + c];
                    Cl[i] = v;
                }
            }
        }
        __syncthreads();
        // A_tt entry (a, a2), both < m
        auto a_entry = [&](int a, int a2) -> T {
            const int s = a / 3, c = a % 3, s2 = a2 / 3, c2 = a2 % 3;
            if (s == s2) return Aself[9 * s + 3 * c + c2];
            if (s2 == s + 1) return Anext[9 * s + 3 * c + c2];
            if (s == s2 + 1) return Anext[9 * s2 + 3 * c2 + c];
            return T(0);
        };
        // Own blocks of S_t = A_tt - (coupling terms).  A term C S^{-1} C^T with
        // couplings C to the two nodes s-1+dn, s+dn of the neighbouring line
        // (dn = 0: line t-1, dn = 1: line t+1) needs, for a 16x16 block with
        // rows R and columns C, S^{-1} only on the node windows of R and C
        // (<= 21 x 21 entries): each wave stages that window of the full
        // symmetric inverse left by the neighbouring line in its own LDS
        // scratch, forms Z = S^{-1}[W(R), .] C_C^T, then subtracts C_R Z.
        if (li > 0 && !f2_wait(cnt, Pf * phase, A, sub, &sh_ok)) return;
        if (mid && nl1 > 0 &&
            !f2_wait(A.counters + F2_COUNTERS * (2 * sub + 1), (uint32_t)(Pf * (NT + 1) * nl1), A, sub, &sh_ok))
            return;
        {
            constexpr int WN = 21;
            T* win = pxr + wv * (WN * WN + WN * 16);                // [WN][WN]
            T* zb = win + WN * WN;                                  // [WN][16]
            constexpr int NWL = (WN * WN + 63) / 64;              // window entries per lane
            // Work items: (block b of this wave, term).  The window loads of the
            // next item are issued before the current item is computed, so the
            // round trip to the neighbour's inverse overlaps the arithmetic.
            const int nbw = nblk > wv ? (nblk - wv + F2_NW - 1) / F2_NW : 0;
            const int nterm = (hup ? 1 : 0) + (hdn ? 1 : 0);
            const int nitem = nbw * nterm;
            auto item = [&](int it, int& b, int& dn, int& r0, int& c0) {
                b = nterm == 2 ? it >> 1 : it;
                dn = nterm == 2 ? (it & 1) : (hup ? 0 : 1);
                int I, J;
                const int blk = wv + F2_NW * b;
                f2_tile_of(blk >> 2, own, I, J);
                r0 = I * TS + 16 * ((blk >> 1) & 1);
                c0 = J * TS + 16 * (blk & 1);
            };
            auto win_rows = [&](int x0, int dn, int& w0, int& n) {
                w0 = max(0, 3 * (x0 / 3 - 1 + dn));
                n = max(0, min(m, 3 * ((x0 + 15) / 3 + dn) + 3) - w0);
            };
            auto issue = [&](int it, T (&w)[NWL]) {
                int b, dn, r0, c0, wr0, nr, wc0, nc;
                item(it, b, dn, r0, c0);
                win_rows(r0, dn, wr0, nr);
                win_rows(c0, dn, wc0, nc);
                const T* S = dn ? Sdn : Sup;
                // every lane loads, with indices clamped into the window (which
                // lies inside the mp x mp inverse: wr0, wc0 <= the block's first
                // row, wr0 + nr, wc0 + nc <= m); the entries outside the window
                // are zeroed where the window is stored.  Branch-free loads whose
                // values are not touched before that keep the compiler's wait
                // counts exact, so the next item's loads stay in flight.
                const int imax = max(nr - 1, 0), jmax = max(nc - 1, 0);
#pragma unroll
                for (int u = 0; u < NWL; ++u) {
                    const int e = lane + 64 * u, i = e / WN, j = e % WN;
                    w[u] = xload(S + (int64_t)(wr0 + min(i, imax)) * mp + wc0 + min(j, jmax));
                }
            };
            V4 v = {T(0), T(0), T(0), T(0)};
            auto a_init = [&](int r0, int c0) {
                const int a2 = c0 + cc;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = r0 + F2T<T>::row(cr, q);
                    v[q] = (a < m && a2 < m) ? a_entry(a, a2) : (a == a2 ? T(1) : T(0));   // identity on the padding
                }
            };
            // subtract the item's term C_R Z, Z = S^{-1}[W(R), W(C)] C_C^T, from v
            auto process = [&](int it, const T (&w)[NWL]) {
                int b, dn, r0, c0, wr0, nr, wc0, nc;
                item(it, b, dn, r0, c0);
                win_rows(r0, dn, wr0, nr);
                win_rows(c0, dn, wc0, nc);
                const T* cf = dn ? Cl : Bl;
                if (nterm == 1 || dn == 0) a_init(r0, c0);         // first term of the block
#pragma unroll
                for (int u = 0; u < NWL; ++u) {
                    const int e = lane + 64 * u, i = e / WN, j = e % WN;
                    if (e < WN * WN) win[e] = (i < nr && j < nc) ? w[u] : T(0);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // Z[i][jc] = sum over the coupled nodes of column c0 + jc; a lane
                // keeps one column jc = lane % 16 (its six coupling coefficients
                // loaded once) and runs over rows i = lane / 16 + 4 u
                {
                    const int jc = lane & 15, a2 = c0 + jc;
                    const bool live = a2 < m;
                    const int nlo = a2 / 3 - 1 + dn, nhi = a2 / 3 + dn;
                    T c2[6];
#pragma unroll
                    for (int g = 0; g < 6; ++g) c2[g] = live ? cf[a2 * 6 + g] : T(0);
                    const bool ulo = live && nlo >= 0, uhi = live && nhi < ms;
                    const int olo = 3 * nlo - wc0, ohi = 3 * nhi - wc0;
#pragma unroll
                    for (int u = 0; u < (WN * 16 + 63) / 64; ++u) {
                        const int i = (lane >> 4) + 4 * u;
                        if (i >= WN) break;
                        T zv = T(0);
                        if (i < nr) {
                            const T* wr = win + i * WN;
#pragma unroll
                            for (int g = 0; g < 3; ++g) {
                                if (ulo) zv = fma(wr[olo + g], c2[g], zv);
                                if (uhi) zv = fma(wr[ohi + g], c2[3 + g], zv);
                            }
                        }
                        zb[i * 16 + jc] = zv;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                // this lane's 4 entries: v -= C_R Z
                const int a2 = c0 + cc;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int a = r0 + F2T<T>::row(cr, q);
                    if (a < m && a2 < m) {
                        const int nlo = a / 3 - 1 + dn, nhi = a / 3 + dn;
                        const T* c1 = cf + a * 6;
                        T u = T(0);
#pragma unroll
                        for (int g = 0; g < 3; ++g) {
                            if (nlo >= 0) u = fma(c1[g], zb[(3 * nlo + g - wr0) * 16 + cc], u);
                            if (nhi < ms) u = fma(c1[3 + g], zb[(3 * nhi + g - wr0) * 16 + cc], u);
                        }
                        v[q] -= u;
                    }
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                if (nterm == 1 || dn == 1) {                          // last term of the block
#pragma unroll
                    for (int q = 0; q < 4; ++q) bscr[(b * 4 + q) * 64 + lane] = v[q];
                }
            };
            if (nterm == 0) {
                // first line of a chain: S_t = A_tt
#pragma unroll 1
                for (int b = 0; b < nbw; ++b) {
                    int I, J;
                    const int blk = wv + F2_NW * b;
                    f2_tile_of(blk >> 2, own, I, J);
                    a_init(I * TS + 16 * ((blk >> 1) & 1), J * TS + 16 * (blk & 1));
#pragma unroll
                    for (int q = 0; q < 4; ++q) bscr[(b * 4 + q) * 64 + lane] = v[q];
                }
            } else {
                // the next item's window is in flight while an item is
                // processed; issues are unconditional (an index past the last
                // item reloads its window, unused) so that the only waits are
                // for the window about to be stored
                T wa[NWL], wb[NWL];
                auto iss = [&](int it, T (&w)[NWL]) { issue(min(it, nitem - 1), w); };
                if (nitem > 0) iss(0, wa);
#pragma unroll 1
                for (int it = 0; it < nitem; it += 2) {
                    iss(it + 1, wb);
                    process(it, wa);
                    iss(it + 2, wa);
                    if (it + 1 < nitem) process(it + 1, wb);
                }
            }
            // blocks of this wave beyond nbw stay zero (never used)
            for (int b = nbw; b < F2_MAXBLK; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) bscr[(b * 4 + q) * 64 + lane] = T(0);
#pragma unroll
            for (int b = 0; b < F2_MAXBLK; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[b][q] = bscr[(b * 4 + q) * 64 + lane];
        }
        __syncthreads();   // LDS (Aself/Anext/Bl) is reused for the exchange column below

        if (rowA == 0 && own.h == 0)                      // hand the first pivot block to the server
            f2_publish_diag<T>(acc, dslot + ((npiv + 1) & 1) * 2 * TSZ, A.epoch + npiv + 1, 0, nblk, own, wv, cr, cc);
        f2_publish<T>(acc, xch + (int64_t)(phase & 1) * NT * TSZ, 0, nblk, own, wv, cr, cc);
        f2_signal(cnt);
        ++phase;

        // ---------- pivot steps -------------------------------------------------
        for (int k = 0; k < NT; ++k, ++phase) {
            int tido = tid;
            asm volatile("" : "+v"(tido));
            fr = tido & 15;
            fk = (tido >> 4) & 3;
            cr = fk;
            cc = fr;
            ++npiv;
            if (!f2_wait(cnt, Pf * phase, A, sub, &sh_ok)) return;
            const T* xb = xch + (int64_t)((phase - 1) & 1) * NT * TSZ;
            const uint64_t* pb = pslot + (npiv & 1) * 2 * TSZ;
            // the column straight into LDS (device-scope 16-byte loads, no
            // registers), while the pivot server is still forming Pi_k:
            // instruction q fills LDS chunks 64 q .. 64 q + 63 of the permuted
            // layout, lane l fetching the chunk that belongs at position 64 q + l
            {
                // E values per 16-byte chunk, CPR chunks per tile row, LPT loads
                // (of 64 chunks) per tile
                constexpr int E = F2T<T>::EPC, CPR = TS / E, LPT = TSZ / (64 * E);
                const int ln = tido & 63, nq = nslots * LPT;
                const int wvu = __builtin_amdgcn_readfirstlane(wv);
#pragma unroll
                for (int u = 0; u < F2_SLOTS * LPT / F2_NW; ++u) {
                    const int q = wvu + F2_NW * u;
                    if (q >= nq) break;
                    const int sl = q / LPT, p = (q % LPT) * 64 + ln;
                    const int J = sl < npar ? own.h + own.sp * sl : ((sl == npar && xtraA) ? rowA : rowB);
                    const int dsl = f2_slot(own, J);
                    const int r = p / CPR, ch = (p % CPR) ^ (r & (CPR - 1));
                    f2_load_lds16(xb + J * TSZ + r * TS + E * ch, colk + (dsl * LPT + q % LPT) * 64 * E);
                }
                __builtin_amdgcn_s_waitcnt(0);
            }
            if (!f2_tpoll<T, T>(pb, A.epoch + npiv, piv, LDPT, A.status, A.status, A.spin_limit, sub, tido)) return;
            __builtin_amdgcn_sched_barrier(0);
            __syncthreads();
            // X_I = S_Ik Pi for the own rows I != k
            for (int rr = 0; rr < nrows; ++rr) {
                const int I = rr == 0 ? rowA : rowB;
                if (I == k) continue;
                // 4 blocks of 16x16 per row, one per wave
                {
                    const int qi = (wv >> 1) & 1, qj = wv & 1;
                    V4 x = {T(0), T(0), T(0), T(0)};
                    #pragma unroll
                    for (int ks = 0; ks < TS / 4; ++ks) {
                        const T a = colk[colk_at_t<T>(f2_slot(own, I), 16 * qi + fr, 4 * ks + fk)];
                        const T b = piv[(4 * ks + fk) * LDPT + 16 * qj + fr];
                        x = F2T<T>::mfma(a, b, x);
                    }
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) xr[rr * LTT + (16 * qi + F2T<T>::row(cr, q)) * LDPT + 16 * qj + cc] = x[q];
                }
            }
            __syncthreads();
            // update own blocks.  When another pivot step follows, the next
            // pivot block goes first (its owner hands it to the pivot server),
            // then the rest of column k+1, which is published and signalled, so
            // that the server and the other ranks' waits overlap the remaining
            // updates.
            const int kn = k + 1;
            const bool own_next = kn < NT && (rowA == kn || rowB == kn) && kn % own.sp == own.h;
#pragma unroll
            for (int pass = 0; pass < 3; ++pass) {
            if (pass == 0 && !own_next) continue;
#pragma unroll
            for (int b = 0; b < F2_MAXBLK; ++b) {
                const int blk = wv + F2_NW * b;
                if (blk >= nblk) continue;
                int I, J;
                f2_tile_of(blk >> 2, own, I, J);
                const int bp = kn >= NT ? 2 : (I == kn && J == kn ? 0 : (I == kn || J == kn ? 1 : 2));
                if (bp != pass) continue;
                const int qi = (blk >> 1) & 1, qj = blk & 1;
                const int rr = (I == rowA) ? 0 : 1;
                if (I != k && J != k) {
                    // S_IJ -= X_I S_kJ.  In product slice ks, lane group fk takes
                    // k = 8 fk + ks (the 32 values of k in any order give the same
                    // sum up to rounding), so that a lane's operands of two slices
                    // are one 16-byte LDS read; all 8 reads are issued before the
                    // 8 products, so only the first product waits on LDS.
                    // (16-byte reads: 2 values each in FP64, 4 in FP32)
                    constexpr int E = F2T<T>::EPC, NR = 8 / E;
                    using VE = T __attribute__((ext_vector_type(E)));
                    VE av[NR], bv[NR];
                    #pragma unroll
                    for (int u = 0; u < NR; ++u) {
                        av[u] = *reinterpret_cast<const VE*>(&xr[rr * LTT + (16 * qi + fr) * LDPT + 8 * fk + E * u]);
                        bv[u] = *reinterpret_cast<const VE*>(
                            &colk[colk_at_t<T>(f2_slot(own, J), 16 * qj + fr, 8 * fk + E * u)]);
                    }
                    V4 v = acc[b];
                    #pragma unroll
                    for (int u = 0; u < NR; ++u)
                        #pragma unroll
                        for (int e = 0; e < E; ++e) v = F2T<T>::mfma(-av[u][e], bv[u][e], v);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2 * NR, 0);   // the LDS reads
                    __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);        // then the 8 products
                    acc[b] = v;
                } else if (I != k) {        // J == k: S_Ik <- X_I
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) acc[b][q] = xr[rr * LTT + (16 * qi + F2T<T>::row(cr, q)) * LDPT + 16 * qj + cc];
                } else if (J != k) {        // I == k: S_kJ <- Pi S_kJ = Pi colk[J]^T
                    V4 v = {T(0), T(0), T(0), T(0)};
                    #pragma unroll
                    for (int ks = 0; ks < TS / 4; ++ks) {
                        const T a = piv[(16 * qi + fr) * LDPT + 4 * ks + fk];
                        const T bb = colk[colk_at_t<T>(f2_slot(own, J), 16 * qj + fr, 4 * ks + fk)];
                        v = F2T<T>::mfma(a, bb, v);
                    }
                    acc[b] = v;
                } else {                    // S_kk <- -Pi
                    #pragma unroll
                    for (int q = 0; q < 4; ++q) acc[b][q] = -piv[(16 * qi + F2T<T>::row(cr, q)) * LDPT + 16 * qj + cc];
                }
                // keep the scheduler from hoisting the operand loads of all
                // blocks at once (register budget)
                __builtin_amdgcn_sched_barrier(0);
            }
            if (pass == 0)
                f2_publish_diag<T>(acc, dslot + ((npiv + 1) & 1) * 2 * TSZ, A.epoch + npiv + 1, kn, nblk, own, wv, cr,
                                cc);
            if (pass == 1 && kn < NT) {
                f2_publish<T>(acc, xch + (int64_t)(phase & 1) * NT * TSZ, kn, nblk, own, wv, cr, cc);
                f2_signal(cnt);
            }
            }
            if (kn >= NT) {
                // ---------- line done: blocks hold -S_t^{-1} ----------------------
                // The blocks go through LDS (the exchange column is free once
                // every wave is past its last update), so that the store code is
                // a loop rather than unrolled over the accumulators and each
                // block's values are a short LDS read away.
                constexpr int NSTG = 12;                 // staged blocks per wave (LDS budget)
                __syncthreads();
                T* stg = colk + wv * NSTG * 256;
#pragma unroll
                for (int b = 0; b < NSTG; ++b)
#pragma unroll
                    for (int q = 0; q < 4; ++q) stg[(b * 4 + q) * 64 + lane] = acc[b][q];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                auto store_block = [&](int b, const T (&vals)[4]) {
                    const int blk = wv + F2_NW * b;
                    int I, J;
                    f2_tile_of(blk >> 2, own, I, J);
                    const int qi = (blk >> 1) & 1, qj = blk & 1;
                    const int q0 = I * (I + 1) / 2 + J;
                    const int64_t toff = ((int64_t)t * d.ntiles + q0) * TSZ;
                    double* tl = Tout + toff;
                    float* tf = reinterpret_cast<float*>(Tout) + toff;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = 16 * qi + F2T<T>::row(cr, q), c = 16 * qj + cc;
                        if (I == J && r < c) continue;           // diagonal tiles: mirror the lower half
                        const T v = -vals[q];
                        if (sizeof(T) == 4 || A.fp32) {
                            tf[r * TS + c] = (float)v;
                            if (I == J) tf[c * TS + r] = (float)v;
                        } else {
                            tl[r * TS + c] = (double)v;
                            if (I == J) tl[c * TS + r] = (double)v;
                        }
                        if (!mid) {                              // the next line of this chain needs it
                            const int ga = I * TS + r, gc = J * TS + c;
                            xstore(Sown + (int64_t)ga * mp + gc, v);
                            xstore(Sown + (int64_t)gc * mp + ga, v);
                        }
                    }
                };
                static_assert(F2_MAXBLK == NSTG + 1, "one block beyond the staged ones");
#pragma unroll 1
                for (int b = 0; b < F2_MAXBLK; ++b) {
                    if (wv + F2_NW * b >= nblk) break;
                    if (b == NSTG) {                     // the last block reuses the first slot
#pragma unroll
                        for (int q = 0; q < 4; ++q) stg[q * 64 + lane] = acc[NSTG][q];
                        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    }
                    const int sb = b < NSTG ? b : 0;
                    T vals[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) vals[q] = stg[(sb * 4 + q) * 64 + lane];
                    store_block(b, vals);
                }
                f2_signal(cnt);
            }
        }
    }
}

template <typename T>
const void* factor2_kernel_of() {
    return (const void*)k_factor2<T>;
}
const void* factor2_kernel(int fp32) { return fp32 ? factor2_kernel_of<float>() : factor2_kernel_of<double>(); }

int launch_line_coeffs(sf_context* c) {
    int maxn = 0;
    for (const auto& d : c->subs) maxn = std::max(maxn, d.nt * d.ms);
    hipLaunchKernelGGL(k_line_coeffs, dim3((maxn + 255) / 256, c->nsub), dim3(256), 0, c->stream, c->d_subs, c->f0,
                       c->alpha, c->factors, c->W, c->H, c->cfg.lambda, 0, (const double*)c->coef);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

// One cooperative factor launch: subdomains [sub0, sub0 + nsub_chunk), or
// the nsub_chunk subdomains listed at sublist (device), in FP64 or FP32
// arithmetic (fp32_arith; the tiles are then stored in FP32), with the pivot
// threshold ptol; rejected pivots flag their subdomain in c->fail_d.
int launch_factor2(sf_context* c, int sub0, int nsub_chunk, int Pf, int fp32_arith, const int32_t* sublist,
                   int lanes, int main_cap, double ptol) {
    FactorArgs a;
    a.subs = c->d_subs;
    a.sub0 = sublist ? 0 : sub0;
    a.nsub = a.sub0 + nsub_chunk;
    a.lanes = lanes;
    a.nmain = std::min(nsub_chunk, main_cap);
    a.pf = Pf;
    a.groups = c->groups;
    a.fp32 = c->cfg.factor_precision != SF_FP64 ? 1 : 0;
    a.f0 = c->f0;
    a.al = c->alpha;
    a.factors = c->factors;
    a.work = c->work;
    a.counters = c->counters;
    a.status = c->status_d;
    a.W = c->W;
    a.H = c->H;
    a.lam = c->cfg.lambda;
    a.spin_limit = c->wait_limit;
    a.ptol = ptol;
    a.fail = c->fail_d;
    a.sublist = sublist;
    // tags must differ from those left in the slots by earlier launches
    a.epoch = c->factor_epoch;
    int maxpiv = 0;
    for (const auto& d : c->subs) maxpiv = std::max(maxpiv, d.nt * d.NT);
    c->factor_epoch += (uint32_t)maxpiv + 4;
    void* args[] = {&a};
    const int L = lanes, per = c->groups * (Pf + 1);
    const int grid = L * ((a.nmain + L - 1) / L) * per + (nsub_chunk - a.nmain) * per;
    if (hipLaunchCooperativeKernel(factor2_kernel(fp32_arith), dim3(grid), dim3(F2_THREADS), args, 0, c->stream) !=
        hipSuccess)
        return SF_ERR_HIP;
    return SF_OK;
}

}  // namespace sfdd

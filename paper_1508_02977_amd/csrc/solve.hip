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
// XCD).  Ranks publish their finished rows as tagged words; the next line
// starts when all P row sets are seen.  No reductions across ranks: P changes
// only the order of the partial sums inside a row.  All waits are bounded: a
// stalled wait raises SF_ERR_DEVICE and every rank exits.
#include <algorithm>

#include "sfdd_internal.h"

namespace sfdd {

#define SF_TRY_SWEEP(x)               \
    do {                              \
        int rc_ = (x);                \
        if (rc_ != SF_OK) return rc_; \
    } while (0)

constexpr int MAXMP = 768;

struct SweepArgs {
    const SubDesc* subs;
    int sub0;               // first subdomain of this launch (mode 0)
    int nsub;               // end of this launch's subdomains (mode 0) ; the single subdomain index (mode 1)
    int lanes;              // subdomains side by side in the grid (8: the ranks of one on one XCD)
    int nmain;              // mode 0: the first nmain subdomains side by side; each later one
                            // takes the next groups x P workgroups (ranks spread over XCDs)
    const double* factors;
    double* work;
    const double* r;        // global residual [B][3][H][W] (mode 0)
    double* U;              // global iterate (mode 0)
    const int32_t* done;    // [B] converged pairs (mode 0)
    const double* b_local;  // local right-hand side (mode 1)
    double* x_local;        // local solution (mode 1)
    DevStatus* status;
    int W, H, mode;
    int groups;             // 1: plain substitution; 2: twisted (both ends towards line kmid)
    uint32_t epoch;         // tag base of this launch (published words carry epoch + phase)
    const uint32_t* epoch_dev;   // if set, the tag base is read here (graph replays)
    long long spin_limit;
};

constexpr int MAXR = 16;   // block rows per rank in the general form

// Tile (I, J) of the block row of symmetric S: lower tile (I,J) if J <= I,
// else the lower tile (J,I) used transposed.  Lane (c, h), c = lane % 16,
// h = lane / 16, holds columns 2c, 2c+1 of rows 8h..8h+7 of the stored tile:
// tv[2i] = T[8h+i][2c], tv[2i+1] = T[8h+i][2c+1] (16-byte loads, a wave
// instruction reads 4 rows of 256 bytes).
__device__ __forceinline__ int32_t tile_lane_offset(int I, int J) {
    const int lane = threadIdx.x & 63;
    const int k = J <= I ? I * (I + 1) / 2 + J : J * (J + 1) / 2 + I;
    return k * TSZ + (8 * (lane >> 4)) * TS + 2 * (lane & 15);
}

__device__ __forceinline__ void load_tile(const double* __restrict__ T, double tv[16]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 v = *reinterpret_cast<const double2*>(T + i * TS);
        tv[2 * i] = v.x;
        tv[2 * i + 1] = v.y;
    }
}
// single-precision tiles: 8-byte loads, same lane layout
__device__ __forceinline__ void load_tile(const float* __restrict__ T, float tv[16]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float2 v = *reinterpret_cast<const float2*>(T + i * TS);
        tv[2 * i] = v.x;
        tv[2 * i + 1] = v.y;
    }
}

// The exchange words: a pair of tagged 64-bit words (low and high half of a
// double) moved as one 16-byte buffer access with the device-scope cache
// policy (sc1: stores write through to memory, loads are not served by a
// possibly stale L1), what relaxed atomics at device scope do, for half the
// memory requests of two 8-byte accesses.  A torn pair is caught by the tags.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ __amdgpu_buffer_rsrc_t words_rsrc(const void* base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
__device__ __forceinline__ u32x4 words_load16(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 16 /* sc1 */);
}
__device__ __forceinline__ void words_store16(u32x4 v, __amdgpu_buffer_rsrc_t r, int byte_off) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, byte_off, 0, 16 /* sc1 */);
}
// The same pair written with the default policy: it stays in the writer's
// XCD L2, where device-scope loads on that XCD see it (loads elsewhere only
// once the line is written back).  Used when every rank of a subdomain runs
// on one XCD; the tags keep any other placement correct, only slower.
__device__ __forceinline__ void words_store16_l2(u32x4 v, __amdgpu_buffer_rsrc_t r, int byte_off) {
    __builtin_amdgcn_raw_buffer_store_b128(v, r, byte_off, 0, 0);
}

// Global-to-LDS copy of 16 bytes per lane (no registers): lane l's bytes land
// at lds + 16 l.  Kept out of the kernel template: its LDS address-space cast
// has no meaning in the host compilation.
__device__ __forceinline__ void sw_dma16(const void* src, void* lds) {
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)lds, 16, 0, 0);
}

// Lane exchanges of the row reductions, kept in the VALU (no LDS crossbar round
// trip).  Within each 16-lane row, DPP gives partners 15 - c (row mirror),
// c ^ 7 inside each half row (half mirror), c ^ 2 and c ^ 1 (quad permutes).
// These pair every lane with one lane of the opposite bit 3, 2, 1, 0 in turn,
// and the four partner maps generate all 16 lanes, so a transpose-reduce over
// them sums each kept row over the whole row group, as xor partners would.
constexpr int DPP_MIRROR = 0x140, DPP_HALF_MIRROR = 0x141, DPP_SWAP2 = 0x4E, DPP_SWAP1 = 0xB1;
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// x plus x of lane ^ 16 (SW = 16) or lane ^ 32 (SW = 32): the permlane swap
// leaves the two halves of every lane pair in the two registers, whose sum is
// the same in both lanes.
template <int SW>
__device__ __forceinline__ double sum_partner(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)b, hi = (unsigned)(b >> 32);
    unsigned l0, l1, h0, h1;
    if constexpr (SW == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = l[0]; l1 = l[1]; h0 = h[0]; h1 = h[1];
    } else {
        static_assert(SW == 32, "lane distance 16 or 32");
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = l[0]; l1 = l[1]; h0 = h[0]; h1 = h[1];
    }
    return __longlong_as_double((long long)(((unsigned long long)h0 << 32) | l0)) +
           __longlong_as_double((long long)(((unsigned long long)h1 << 32) | l1));
}
// Transpose-reduce of 8 row partials p[8] over the 16 lanes of a row group:
// lane c ends with row 4 b3 + 2 b2 + b1 (bits of c) in p[0].
__device__ __forceinline__ void row_group_reduce(double p[8], int c) {
    const int b3 = (c >> 3) & 1, b2 = (c >> 2) & 1, b1 = (c >> 1) & 1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double keep = b3 ? p[q + 4] : p[q], send = b3 ? p[q] : p[q + 4];
        p[q] = keep + dpp_partner<DPP_MIRROR>(send);
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const double keep = b2 ? p[q + 2] : p[q], send = b2 ? p[q] : p[q + 2];
        p[q] = keep + dpp_partner<DPP_HALF_MIRROR>(send);
    }
    {
        const double keep = b1 ? p[1] : p[0], send = b1 ? p[0] : p[1];
        p[0] = keep + dpp_partner<DPP_SWAP2>(send);
    }
    p[0] += dpp_partner<DPP_SWAP1>(p[0]);
}

// y_I += (tile) z_J for one tile of the block row, into the wave's row buffer y[32].
template <typename TT>
__device__ __forceinline__ void tile_apply(const TT tv[16], int I, int J, const double* z, double* y) {
    const int lane = threadIdx.x & 63;
    const int c = lane & 15, h = lane >> 4;
    if (J >= I) {
        // stored (J, I) used transposed, or the symmetric diagonal tile:
        // y_I[col] += sum_r T[r][col] zJ[r] over this lane's rows, then over the 4 row groups
        const double* zr = z + J * TS + 8 * h;
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            s0 = fma((double)tv[2 * i], zr[i], s0);
            s1 = fma((double)tv[2 * i + 1], zr[i], s1);
        }
        s0 = sum_partner<32>(sum_partner<16>(s0));
        s1 = sum_partner<32>(sum_partner<16>(s1));
        if (h == 0) {
            y[2 * c] += s0;
            y[2 * c + 1] += s1;
        }
    } else {
        // stored (I, J): y_I[r] += sum_col T[r][col] zJ[col]; 8 row partials per
        // lane reduced over the 16 lanes of the row group (transpose-reduce:
        // xor 8, 4, 2, then 1)
        const double z0 = z[J * TS + 2 * c], z1 = z[J * TS + 2 * c + 1];
        double p[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) p[i] = fma((double)tv[2 * i], z0, (double)tv[2 * i + 1] * z1);
        row_group_reduce(p, c);
        if ((c & 1) == 0) y[8 * h + (c >> 1)] += p[0];
    }
}

// i-th own block row of rank `rank` among P ranks: rows are dealt in
// boustrophedon order (0..P-1, then P-1..0, ...), so with NT <= 2P a rank owns
// the pair (r, 2P-1-r) and every rank meets about the same number of tiles
// that it applies directly and transposed.  Row numbers increase with i.
__device__ __forceinline__ int own_row(int i, int rank, int P) {
    return 2 * P * (i >> 1) + ((i & 1) ? 2 * P - 1 - rank : rank);
}

// Twisted sweep.  The lines of a subdomain are eliminated from both ends
// towards the middle line k (the factor stores S_t^{-1} of the top chain for
// t < k, of the bottom chain for t > k and of the middle line for t = k):
//   top    (group 0):  w_t = S_t^{-1} (r_t - B_t w_{t-1}),          t = 0..k-1
//   bottom (group 1):  w_t = S_t^{-1} (r_t - B_{t+1}^T w_{t+1}),    t = nt-1..k+1
//   middle (both):     x_k = S_k^{-1} (r_k - B_k w_{k-1} - B_{k+1}^T w_{k+1})
//   top back:          x_t = w_t - S_t^{-1} B_{t+1}^T x_{t+1},      t = k-1..0
//   bottom back:       x_t = w_t - S_t^{-1} B_t x_{t-1},            t = k+1..nt-1
// so a sweep takes 2 max(k, nt-1-k) + 1 dependent phases instead of 2 nt - 1.
// With one group (k = nt - 1) this is the plain forward/backward substitution.
// Each group has P ranks (workgroups); both groups compute the middle line
// (group 0 stores it).
//
// Within a rank, waves 0..NW-2 ("tile waves") hold its tiles of the line
// matrix and the right-hand side terms; the last wave ("control wave") does
// the latency-critical traffic: it gathers the rows the phase needs, finishes
// and publishes this rank's rows.  Global loads of a wave complete in order,
// so keeping the tile loads of the next line (issued by the tile waves one
// phase ahead) off the control wave keeps its polls short.  With FP64 tiles
// each slot is reloaded right after its products, so the stream runs under
// the compute and is mostly done when the control wave polls; with FP32 tiles
// (half the bytes) the loads follow the products.  All addressing is set up
// in registers; nothing inside the phase loop loads an address from memory
// (such a load would drain the load queue).
// Workgroup g is dispatched to XCD g % 8; the ranks of subdomain i are the
// workgroups g with g % 8 == i % 8, so the tiles that two ranks of one
// subdomain both read are shared through one L2.  Correctness does not depend
// on the placement: the exchange uses device-scope accesses.
template <typename TT, int RMAX, int PF, int LMAX, int NWV>
__global__ void __launch_bounds__(64 * NWV) k_sweep(SweepArgs A) {
    constexpr int NTHR = 64 * NWV;
    constexpr int NW = NWV;
    constexpr int NWT = NW - 1;                    // tile waves
    constexpr int CW0 = NWT * 64;                  // first thread of the control wave
    constexpr int NRC = (RMAX * TS + 63) / 64;     // own rows per control lane
    // rows of z per tile-wave thread: general form, all rows over the tile
    // threads; fast form, the 32 (PF / 2) rows of the wave's column blocks
    constexpr bool FAST = RMAX <= 2;
    constexpr int PH = PF / RMAX;                  // fast form: tile slots per own row
    constexpr int RPT = FAST ? (32 * PH + 63) / 64 : (LMAX + CW0 - 1) / CW0;
    __shared__ double z[LMAX];
    __shared__ double vup[LMAX];                   // vector of the line above (t - 1)
    __shared__ double vdn[LMAX];                   // vector of the line below (t + 1)
    __shared__ double yw[NWT][RMAX * TS];
    __shared__ int sh_ok;
    // Staged tiles (FP32 tiles, fast forms): the next line's tiles are copied
    // from memory straight into LDS at the start of a phase (NWT x PF tiles,
    // 112 KB per workgroup; the fast forms run one workgroup per CU anyway),
    // where they stream in while the phase synchronises.  A tile takes 4 copies
    // of 16 bytes per lane (copy j: lane l the row 8 j + l / 8, columns
    // 4 (l % 8) .. + 3), so the staged tile is the stored tile, row-major.
    constexpr bool STAGE = FAST && sizeof(TT) == 4;
    __shared__ __attribute__((aligned(16))) TT stg[STAGE ? NWT * PF * TSZ : 1];

    const int mode = A.mode, G = A.groups;
    int sub, grp, rank;
    bool side_by_side = false;                     // with 8 lanes: every rank of sub on one XCD
    {
        const int P0 = A.subs[0].P, per = G * P0;
        if (mode == 1) {
            const int x = blockIdx.x % A.lanes, slot = blockIdx.x / A.lanes;
            if (x != 0) return;                        // idle slot
            sub = A.nsub;
            grp = slot / P0;
            rank = slot % P0;
        } else {
            const int mainwg = A.lanes * ((A.nmain + A.lanes - 1) / A.lanes) * per;
            int local, within;
            if ((int)blockIdx.x < mainwg) {
                const int x = blockIdx.x % A.lanes, slot = blockIdx.x / A.lanes;
                local = x + A.lanes * (slot / per);
                within = slot % per;
                if (local >= A.nmain) return;          // idle slot
                side_by_side = true;
            } else {
                const int b = (int)blockIdx.x - mainwg;
                local = A.nmain + b / per;
                within = b % per;
            }
            sub = A.sub0 + local;
            grp = within / P0;
            rank = within % P0;
            if (sub >= A.nsub) return;                 // idle slot
        }
    }
    const SubDesc d = A.subs[sub];
    if (mode == 0 && A.done[d.pair]) return;   // uniform over the subdomain's ranks
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const bool ctl = wv == NWT;
    const int P = d.P, m = d.m, mp = d.mp, ms = d.ms, nt = d.nt, NT = d.NT, km = d.kmid;
    int R = 0;                                     // own block rows: own_row(i), i < R
    while (R < RMAX && own_row(R, rank, P) < NT) ++R;
    if (R == 0) return;                            // no rows (P > NT): nothing to do
    const int ntw = R * NT;                        // tiles per phase for this rank
    const int nrow = R * TS;                       // rows finished by this rank
    const int L = grp == 0 ? km : nt - 1 - km;     // lines of this group's chain
    const int nphase = 2 * L + 1;
    const int64_t nn = (int64_t)A.W * A.H;
    const int64_t tstride = (int64_t)d.ntiles * TSZ;       // tiles of one line
    const TT* __restrict__ Tb = reinterpret_cast<const TT*>(A.factors + d.foff);   // tiles of double or float
    const double* __restrict__ Bb = A.factors + d.boff;
    double* __restrict__ wst = A.work + d.woff;            // w_t, then x_t, of this rank's rows
    // published rows: per group [3][mp] pairs of 64-bit words (tag << 32 | half
    // of a double); slots 0/1 by phase parity, slot 2 for the last forward line
    uint64_t* __restrict__ pub = reinterpret_cast<uint64_t*>(A.work + d.poff);
    const __amdgpu_buffer_rsrc_t pubr = words_rsrc(pub, 12 * mp * 8);
    // 8 subdomains side by side: workgroup g runs on XCD g mod 8, so all
    // ranks of a subdomain share one L2 and the published words can stay there
    const bool pub_l2 = A.lanes == 8 && side_by_side;
    DevStatus* st = A.status;
    const long long spin = A.spin_limit;
    const uint32_t epoch = A.epoch_dev ? *A.epoch_dev : A.epoch;
    auto tag_of = [&](int g, int q) -> uint32_t { return epoch + 2u * (uint32_t)q + (uint32_t)g; };
    auto slot_of = [&](int g, int q) -> const uint64_t* {
        const int Lg = g == 0 ? km : nt - 1 - km;
        const int sl = q == Lg - 1 ? 2 : (q & 1);
        return pub + ((int64_t)g * 3 + sl) * 2 * mp;
    };
    // phase q -> line, kind, couplings
    auto line_of = [&](int q) -> int {
        if (q < L) return grp == 0 ? q : nt - 1 - q;
        if (q == L) return km;
        return grp == 0 ? 2 * L - q : km + (q - L);
    };

    // local unknown a of line t sits at global index gbase(a) + t * gstep
    const int64_t gstep = d.cols ? 1 : (int64_t)A.W;
    auto gbase = [&](int a) -> int64_t {
        const int s = a / 3, c = a % 3;
        const int x = d.cols ? d.bx0 : d.bx0 + s, y = d.cols ? d.by0 + s : d.by0;
        return ((int64_t)d.pair * 3 + c) * nn + (int64_t)y * A.W + x;
    };
    // Rows of z that this thread forms.  Fast form: a tile wave forms exactly
    // the rows it consumes (its column blocks wv + NWT i), so no workgroup
    // barrier separates z from the products; general form: rows tid + CW0 j.
    static_assert(!FAST || (64 * RPT >= 32 * PH && PF % RMAX == 0), "fast form: z rows of a wave = its column blocks");
    // (The thread index is passed through an empty asm statement where rows
    // are formed inside the phase loop, so that the compiler recomputes the
    // few integer operations of their addresses instead of keeping a set of
    // 64-bit addresses live across the whole loop.)
    constexpr bool OPAQUE = sizeof(TT) == 8;       // FP64 tiles leave few spare registers
    auto zrow = [&](int j) -> int {
        int tx = tid;
        if constexpr (OPAQUE) asm volatile("" : "+v"(tx));
        if constexpr (FAST) {
            const int k = (tx & 63) + 64 * j;
            if (k >= 32 * PH) return LMAX;                  // no row (a lane beyond the wave's blocks)
            return ((tx >> 6) + NWT * (k >> 5)) * TS + (k & 31);
        } else {
            return tx + CW0 * j;
        }
    };
    // right-hand side of row a of line t (FP32 tiles: base pointers kept per row)
    const int64_t rstep = mode == 1 ? m : gstep;
    const double* __restrict__ rbase[OPAQUE ? 1 : RPT];
    if constexpr (!OPAQUE) {
#pragma unroll
        for (int j = 0; j < RPT; ++j) {
            const int a = zrow(j);
            rbase[j] = mode == 1 ? A.b_local + a : A.r + (a < m ? gbase(a) : 0);
        }
    }
    auto rsrc = [&](int j, int a, int t) -> const double* {
        if constexpr (OPAQUE)
            return mode == 1 ? A.b_local + a + (int64_t)t * rstep : A.r + gbase(a) + (int64_t)t * rstep;
        else
            return rbase[j] + (int64_t)t * rstep;
    };
    // this thread's prefetched tiles (fixed for all lines): offsets inside a line
    // Fast form (RMAX <= 2 rows per rank, NT <= NWT PH, PH = PF / RMAX): slot p
    // holds tile (row p / PH, column wv + NWT (p % PH)), so a wave's tiles of one
    // row are fixed and the row partials stay in registers until one reduction
    // per row.  General form: slot p holds the tile qt = wv + NWT p of the
    // rank's row-major list.
    constexpr bool RELOAD = FAST && sizeof(TT) == 8;   // tile slots reloaded right after their products
    auto slot_ok = [&](int p) -> bool {
        if constexpr (FAST) return p / PH < R && wv + NWT * (p % PH) < NT;
        else return wv + NWT * p < ntw;
    };
    int32_t toff[PF];                              // < ntiles * TSZ elements
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        if constexpr (FAST) {
            toff[p] = slot_ok(p) ? tile_lane_offset(own_row(p / PH, rank, P), wv + NWT * (p % PH)) : 0;
        } else {
            const int qt = min(wv + NWT * p, ntw - 1);
            toff[p] = tile_lane_offset(own_row(qt / NT, rank, P), qt % NT);
        }
    }
    // own rows of the control lanes
    int crow[NRC];
#pragma unroll
    for (int i = 0; i < NRC; ++i) {
        const int k = tid - CW0 + 64 * i;
        crow[i] = k < nrow ? own_row(k / TS, rank, P) * TS + k % TS : -1;
    }

    TT pre[PF][16];
    // prefetched right-hand side and coupling coefficients of this thread's
    // rows: pb holds the up coefficients when the phase has an up term, else
    // the down ones (the middle phase, which has both, reads the down ones in z)
    double pr[RPT], pb[RPT][6];
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
        pr[j] = 0.0;
#pragma unroll
        for (int e = 0; e < 6; ++e) pb[j][e] = 0.0;
    }
    // B_{t+1}^T row a (nodes s, s+1 of line t+1) from the stored rows of B_{t+1}
    auto dn_coeffs = [&](int t, int a, double* c6) {
        const int zs = a / 3, ze = a % 3;
        const double* Bt = Bb + (int64_t)(t + 1) * m * 6;
#pragma unroll
        for (int c = 0; c < 3; ++c) c6[c] = Bt[(int64_t)(3 * zs + c) * 6 + 3 + ze];
#pragma unroll
        for (int c = 0; c < 3; ++c) c6[3 + c] = zs + 1 < ms ? Bt[(int64_t)(3 * (zs + 1) + c) * 6 + ze] : 0.0;
    };
    // coupling terms of phase q: up = B_t (rows of line t, nodes s-1, s of
    // line t-1), dn = B_{t+1}^T (nodes s, s+1 of line t+1)
    auto has_up = [&](int q, int t) -> bool {
        return (q < L) ? (grp == 0 && t > 0) : (q == L ? t > 0 : grp == 1);
    };
    auto has_dn = [&](int q, int t) -> bool {
        return (q < L) ? (grp == 1 && t < nt - 1) : (q == L ? t < nt - 1 : grp == 0);
    };
    auto prefetch = [&](int q, bool tiles) {        // tile waves
        const int t = line_of(q);
        const bool hu = has_up(q, t), hd = has_dn(q, t);
#pragma unroll
        for (int j = 0; j < RPT; ++j) {             // z terms first: needed earlier
            const int a = zrow(j);
            if (a < m) {
                if (q <= L) pr[j] = *rsrc(j, a, t);
                if (hu) {
                    const double* cf = Bb + ((int64_t)t * m + a) * 6;
#pragma unroll
                    for (int e = 0; e < 6; ++e) pb[j][e] = cf[e];
                } else if (hd) {
                    dn_coeffs(t, a, pb[j]);
                }
            }
        }
        if (!tiles) return;
        const TT* Tl = Tb + (int64_t)t * tstride;
#pragma unroll
        for (int p = 0; p < PF; ++p)
            if (slot_ok(p)) load_tile(Tl + toff[p], pre[p]);
    };
    // staged slots: copy the tiles of phase q into LDS / from LDS into registers
    const int lanepart = (8 * (lane >> 4)) * TS + 2 * (lane & 15);   // of tile_lane_offset
    auto stage_issue = [&](int q) {
        const TT* Tl = Tb + (int64_t)line_of(q) * tstride;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            if (!slot_ok(p)) continue;
            const int tb = toff[p] - lanepart;                      // the tile's first element
            TT* dst = stg + (wv * PF + p) * TSZ;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sw_dma16(Tl + tb + (8 * j + (lane >> 3)) * TS + 4 * (lane & 7), dst + j * 256);
        }
    };
    auto stage_read = [&]() {
        const int h = lane >> 4, c = lane & 15;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
            if (!slot_ok(p)) continue;
            const TT* src = stg + (wv * PF + p) * TSZ + h * 256 + 2 * (c & 1);
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                // row 8h + i, columns 2c, 2c + 1: copy h, lane 8 i + c / 2, half c % 2
                const float2 v = *reinterpret_cast<const float2*>(src + 4 * (8 * i + (c >> 1)));
                pre[p][2 * i] = v.x;
                pre[p][2 * i + 1] = v.y;
            }
        }
    };
    // control wave: poll the published words of (group g, phase q) into dst,
    // at most GMAX words per lane in flight (registers), group after group
    auto gather = [&](int g, int q, double* dst) -> int {
        const uint32_t tag = tag_of(g, q);
        const int pb0 = (int)(slot_of(g, q) - pub) * 8;    // byte offset of the slot
        constexpr int NG = LMAX / 64, GMAX = 6;
        long long n = 0;
#pragma unroll 1
        for (int u0 = 0; u0 < NG; u0 += GMAX) {
            constexpr int GW = NG < GMAX ? NG : GMAX;
            uint64_t lo[GW], hi[GW];
            unsigned pending = 0;
#pragma unroll
            for (int v = 0; v < GW; ++v)
                if (u0 + v < NG && lane + 64 * (u0 + v) < mp) pending |= 1u << v;
            while (pending) {
#pragma unroll
                for (int v = 0; v < GW; ++v)
                    if (pending & (1u << v)) {
                        const int a = lane + 64 * (u0 + v);
                        const u32x4 w = words_load16(pubr, pb0 + 16 * a);
                        lo[v] = ((uint64_t)w[1] << 32) | w[0];
                        hi[v] = ((uint64_t)w[3] << 32) | w[2];
                    }
#pragma unroll
                for (int v = 0; v < GW; ++v)
                    if ((pending & (1u << v)) && (uint32_t)(lo[v] >> 32) == tag && (uint32_t)(hi[v] >> 32) == tag) {
                        dst[lane + 64 * (u0 + v)] =
                            __longlong_as_double((long long)((hi[v] << 32) | (lo[v] & 0xffffffffull)));
                        pending &= ~(1u << v);
                    }
                if (!pending) break;
                if (++n > spin ||
                    __hip_atomic_load(&st->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == SF_ERR_DEVICE)
                    return 0;
                __builtin_amdgcn_s_sleep(1);
            }
        }
        return 1;
    };
    double pw[NRC];
#pragma unroll
    for (int i = 0; i < NRC; ++i) pw[i] = 0.0;

    for (int i = tid; i < NWT * RMAX * TS; i += NTHR) (&yw[0][0])[i] = 0.0;
    if (!ctl) {
        prefetch(0, true);
        if constexpr (STAGE)
            if (nphase > 1) stage_issue(1);
    }
    // Phase structure (B = workgroup barrier):
    //   control wave: [gather(q)] B z B  .  B [finish, publish(q)]
    //   tile waves:              B z B [compute(q)] B [prefetch(q+1)]
    //   (FP64 tiles: the tiles of q+1 are loaded inside compute(q), slot by slot;
    //    staged FP32 tiles: phase q starts by taking its tiles from LDS and
    //    copying those of q+1 there)
    // Rows are exchanged as tagged 64-bit words (32-bit tag, 32-bit half of a
    // double): a reader polls the words it needs until both halves carry the
    // tag of the wanted phase, so one memory round trip both synchronises and
    // transfers the data; no separate flag, counter or store acknowledgement.
    __syncthreads();
    for (int q = 0; q < nphase; ++q) {
        const int t = line_of(q);
        const bool back = q > L;
        const bool up = has_up(q, t), dn = has_dn(q, t);
        if constexpr (STAGE) {
            if (!ctl && q > 0) {
                // this phase's tiles, copied into LDS during the previous phase
                // (vmcnt 0: the copies have landed, and so have the vectors
                // prefetched for this phase), into registers; once those LDS
                // reads are done (lgkmcnt 0) the slots take the next phase's
                // tiles, which stream in under this phase's synchronisation
                __builtin_amdgcn_s_waitcnt(0x0F70);
                stage_read();
                __builtin_amdgcn_s_waitcnt(0xC07F);
                if (q + 1 < nphase) stage_issue(q + 1);
            }
        }
        if (up || dn) {
            if (ctl) {
                int ok = 1;
                if (q == L) {                      // middle: last forward vectors of both chains
                    if (up) ok = gather(0, km - 1, vup);
                    if (dn && ok) ok = gather(1, nt - 2 - km, vdn);
                } else {
                    ok = gather(grp, q - 1, up ? vup : vdn);
                }
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
            if (!sh_ok) {
                if constexpr (STAGE) __builtin_amdgcn_s_waitcnt(0);   // no copy into LDS left in flight
                return;
            }
        }
        // z: forward / middle r_t - (coupling terms); backward the coupling term
        if (!ctl) {
#pragma unroll
            for (int j = 0; j < RPT; ++j) {
                const int a = zrow(j), zs = a / 3;
                if (a >= mp) break;
                double v = 0.0;
                if (a < m) {
                    double cu = 0.0;
                    if (up) {
                        if (zs > 0)
#pragma unroll
                            for (int e = 0; e < 3; ++e) cu = fma(pb[j][e], vup[3 * (zs - 1) + e], cu);
#pragma unroll
                        for (int e = 0; e < 3; ++e) cu = fma(pb[j][3 + e], vup[3 * zs + e], cu);
                    }
                    if (dn) {
                        double cd[6];
                        if (up) dn_coeffs(t, a, cd);                 // middle phase only
                        else {
#pragma unroll
                            for (int e = 0; e < 6; ++e) cd[e] = pb[j][e];
                        }
#pragma unroll
                        for (int e = 0; e < 3; ++e) cu = fma(cd[e], vdn[3 * zs + e], cu);
                        if (zs + 1 < ms)
#pragma unroll
                            for (int e = 0; e < 3; ++e) cu = fma(cd[3 + e], vdn[3 * (zs + 1) + e], cu);
                    }
                    v = back ? cu : pr[j] - cu;
                }
                z[a] = v;
            }
        }
        if constexpr (FAST) {
            // each tile wave reads only its own rows of z
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        } else {
            __syncthreads();
        }
        if (!ctl) {
            // this rank's block rows
            if constexpr (FAST) {
                // per own row i: direct partials dp[k] of rows 8h+k and
                // transposed partials tp0, tp1 of columns 2c, 2c+1, summed over
                // this wave's tiles of the row, then one reduction per row
                const int c = lane & 15, h = lane >> 4;
#pragma unroll
                for (int i = 0; i < RMAX; ++i) {
                    if (i >= R) break;
                    const int I = own_row(i, rank, P);
                    double d[8], s0 = 0.0, s1 = 0.0;
#pragma unroll
                    for (int k = 0; k < 8; ++k) d[k] = 0.0;
#pragma unroll
                    for (int u = 0; u < PH; ++u) {
                        const int p = i * PH + u;
                        if (!slot_ok(p)) continue;
                        const int J = wv + NWT * u;
                        if (J >= I) {
                            const double* zr = z + J * TS + 8 * h;
#pragma unroll
                            for (int k = 0; k < 8; ++k) {
                                s0 = fma((double)pre[p][2 * k], zr[k], s0);
                                s1 = fma((double)pre[p][2 * k + 1], zr[k], s1);
                            }
                        } else {
                            const double z0 = z[J * TS + 2 * c], z1 = z[J * TS + 2 * c + 1];
#pragma unroll
                            for (int k = 0; k < 8; ++k)
                                d[k] = fma((double)pre[p][2 * k], z0, fma((double)pre[p][2 * k + 1], z1, d[k]));
                        }
                        // FP64 tiles: the slot is free, so its tile of the next
                        // line streams in under the rest of this phase (with FP32
                        // tiles the stream is short enough to follow the products)
                        if constexpr (RELOAD)
                            if (q + 1 < nphase) load_tile(Tb + (int64_t)line_of(q + 1) * tstride + toff[p], pre[p]);
                    }
                    double* y = &yw[wv][i * TS];
                    row_group_reduce(d, c);
                    s0 = sum_partner<32>(sum_partner<16>(s0));
                    s1 = sum_partner<32>(sum_partner<16>(s1));
                    if ((c & 1) == 0) y[8 * h + (c >> 1)] = d[0];   // yw is zero here
                    if (h == 0) {
                        y[2 * c] += s0;
                        y[2 * c + 1] += s1;
                    }
                }
            } else {
#pragma unroll
                for (int p = 0; p < PF; ++p) {
                    const int qt = wv + NWT * p;
                    if (qt < ntw) tile_apply(pre[p], own_row(qt / NT, rank, P), qt % NT, z, &yw[wv][(qt / NT) * TS]);
                }
                for (int qt = wv + NWT * PF; qt < ntw; qt += NWT) {
                    const int i = qt / NT, I = own_row(i, rank, P);
                    TT tv[16];
                    load_tile(Tb + (int64_t)t * tstride + tile_lane_offset(I, qt % NT), tv);
                    tile_apply(tv, I, qt % NT, z, &yw[wv][i * TS]);
                }
            }
        }
        __syncthreads();
        if (!ctl) {
            // (with RELOAD the tile slots have already been reloaded for the next line)
            if (q + 1 < nphase) prefetch(q + 1, !RELOAD && !STAGE);
        } else {
            // finish and publish this rank's rows; keep them; prefetch w
            const uint64_t tag = (uint64_t)tag_of(grp, q) << 32;
            uint64_t* pout = const_cast<uint64_t*>(slot_of(grp, q));
            const bool keep = !(q == L && grp == 1);           // group 0 stores the middle line
            double* wt = wst + (int64_t)t * mp;
#pragma unroll
            for (int i = 0; i < NRC; ++i) {
                const int k = tid - CW0 + 64 * i;
                if (crow[i] >= 0) {
                    double y = 0.0;
                    if constexpr (FAST) {
                        // every tile wave rewrites all its rows each phase
#pragma unroll
                        for (int w = 0; w < NWT; ++w) y += yw[w][k];
                    } else {
                        for (int w = 0; w < NWT; ++w) {
                            y += yw[w][k];
                            yw[w][k] = 0.0;
                        }
                    }
                    if (back) y = pw[i] - y;               // x_t = w_t - S_t^{-1} v
                    const uint64_t bits = (uint64_t)__double_as_longlong(y);
                    const uint32_t tg = (uint32_t)(tag >> 32);
                    const u32x4 w = {(uint32_t)bits, tg, (uint32_t)(bits >> 32), tg};
                    if (pub_l2) words_store16_l2(w, pubr, (int)(pout - pub) * 8 + 16 * crow[i]);
                    else words_store16(w, pubr, (int)(pout - pub) * 8 + 16 * crow[i]);
                    if (keep) wt[crow[i]] = y;                     // w_t or x_t
                }
            }
            if (q + 1 < nphase && q + 1 > L) {
                const double* wn = wst + (int64_t)line_of(q + 1) * mp;   // w of the next backward line
#pragma unroll
                for (int i = 0; i < NRC; ++i) pw[i] = crow[i] >= 0 ? wn[crow[i]] : 0.0;
            }
        }
    }
    // U[O_i] += x on the owned nodes of this rank's rows and of this group's
    // lines: group 0 lines 0..k, group 1 lines k+1..nt-1
    __syncthreads();
    const int t0 = grp == 0 ? 0 : km + 1, t1 = grp == 0 ? km + 1 : nt;
    for (int i = tid; i < (t1 - t0) * nrow; i += NTHR) {
        const int t = t0 + i / nrow, k = i % nrow;
        const int a = own_row(k / TS, rank, P) * TS + k % TS;
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

// Launch forms.  General: 4 waves (3 tile waves; one wave per SIMD, 512
// registers each), any number of block rows per rank.  Fast forms, all of a
// phase's tiles in registers (8 waves: 7 tile waves of 4 tile slots, within
// 256 VGPRs, two waves per SIMD): at most two block rows per rank and lines
// up to 448 (NT <= 14), or one block row per rank and lines up to 768.
// FP64 or FP32 tiles.
constexpr int GEN_WAVES = 4;
constexpr int FAST2_LMAX = 448, FAST1_LMAX = 768;
template <typename TT>
const void* sweep_kernel_of(int form) {
    if (form == SWEEP_FAST2) return (const void*)k_sweep<TT, 2, 4, FAST2_LMAX, 8>;
    if (form == SWEEP_FAST1) return (const void*)k_sweep<TT, 1, 4, FAST1_LMAX, 8>;
    return (const void*)k_sweep<TT, MAXR, 4, MAXMP, GEN_WAVES>;
}
const void* sweep_kernel(int form, int fp32) {
    return fp32 ? sweep_kernel_of<float>(form) : sweep_kernel_of<double>(form);
}
int sweep_threads(int form) { return form == SWEEP_GENERAL ? 64 * GEN_WAVES : 512; }

// The form of the current shape: the fast forms when every rank owns at
// most two block rows of lines up to 448 or one block row of any line.
int sweep_form(const sf_context* c) {
    int maxmp = 0;
    for (const auto& d : c->subs) maxmp = std::max(maxmp, d.mp);
    if (c->sweep_rows <= 2 && maxmp <= FAST2_LMAX) return SWEEP_FAST2;
    if (c->sweep_rows <= 1 && maxmp <= FAST1_LMAX) return SWEEP_FAST1;
    return SWEEP_GENERAL;
}

uint32_t sweep_epoch_step(const sf_context* c) {
    int maxph = 0;
    for (const auto& d : c->subs) maxph = std::max(maxph, 2 * d.nt);
    return 2u * (uint32_t)maxph + 4;
}

int launch_sweep(sf_context* c, double* U, const double* r, int single_sub, const double* b_local, double* x_local) {
    SweepArgs a;
    a.subs = c->d_subs;
    a.factors = c->factors;
    a.work = c->work;
    a.r = r;
    a.U = U;
    a.done = c->done_d;
    a.b_local = b_local;
    a.x_local = x_local;
    a.status = c->status_d;
    a.W = c->W;
    a.H = c->H;
    a.mode = single_sub >= 0 ? 1 : 0;
    a.groups = c->groups;
    a.spin_limit = c->wait_limit;
    // tags must differ from every tag left in the exchange buffers by earlier
    // launches: advance by more than the tags of one sweep (2 per phase).  The
    // launches of one sweep's chunks share the tag base: their subdomains'
    // exchange buffers are disjoint.  While a graph is captured the kernel
    // reads the tag base from the device counter that the graph advances
    // after every sweep.
    a.epoch = c->sweep_epoch;
    a.epoch_dev = c->graph_capture ? c->gepoch_d : nullptr;
    c->sweep_epoch += sweep_epoch_step(c);
    const int ranks = c->groups * c->maxP;
    const int form = sweep_form(c);
    const void* kern = sweep_kernel(form, c->cfg.factor_precision != SF_FP64);
    const int threads = sweep_threads(form);
    void* args[] = {&a};
    // An ordinary launch, captured or not: the grid fits the co-resident
    // capacity measured at creation, so every workgroup becomes resident once
    // the work ahead of it on the device drains (the sweeps of other contexts
    // do not overlap: the calls that launch sweeps hold a per-device lock),
    // and every wait is bounded.  A cooperative launch guarantees the same
    // residency at a higher cost per launch (283 against 279 ms per step of
    // the 640x480 workload).
    auto launch = [&](int grid) -> int {
        if (hipLaunchKernel(kern, dim3(grid), dim3(threads), args, 0, c->stream) != hipSuccess) return SF_ERR_HIP;
        return SF_OK;
    };
    if (single_sub >= 0) {
        a.sub0 = 0;
        a.nsub = single_sub;
        a.lanes = 1;
        a.nmain = 1;
        return launch(ranks);
    }
    // chunks of subdomains whose ranks fit co-resident, one launch each: the
    // first side by side in groups of L, the rest on contiguous workgroups
    const int L = c->sweep_lanes, chunk = c->sweep_chunk;
    a.lanes = L;
    for (int s0 = 0; s0 < c->nsub; s0 += chunk) {
        const int n = std::min(chunk, c->nsub - s0);
        a.sub0 = s0;
        a.nsub = s0 + n;
        a.nmain = std::min(n, c->sweep_main);
        SF_TRY_SWEEP(launch(L * ((a.nmain + L - 1) / L) * ranks + (n - a.nmain) * ranks));
    }
    return SF_OK;
}

}  // namespace sfdd

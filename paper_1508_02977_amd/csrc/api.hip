// C ABI of the sfdd library: context, geometry, entry points.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <optional>

#include "sfdd_internal.h"
#include "factor2_layout.h"

using sfdd::SubDesc;

namespace {

constexpr int ST_CREATED = 0, ST_ASSEMBLED = 1, ST_FACTORED = 2;
constexpr int PENDING_ASSEMBLE = 1, PENDING_FACTOR = 2;
constexpr int MAX_LINE = 768;        // largest padded line matrix (3 x the shorter box side, rounded up to 32)

template <class T>
int dalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    if (hipMalloc((void**)p, count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return SF_ERR_OOM;
    }
    return SF_OK;
}

#define SF_TRY(x)                    \
    do {                             \
        int rc_ = (x);               \
        if (rc_ != SF_OK) return rc_; \
    } while (0)
#define SF_HIP(x)                                   \
    do {                                            \
        if ((x) != hipSuccess) return SF_ERR_HIP;   \
    } while (0)

__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_zero_status_api(sfdd::DevStatus* st) {
    st->code = 0;
    st->sub = -1;
    st->row = -1;
}

// Device counters of a graph-replayed Schwarz loop: iteration index and sweep
// tag base, set once, then advanced by the graph after every sweep.
__global__ void k_graph_init(int32_t* k, uint32_t* epoch, uint32_t e0) {
    *k = 0;
    *epoch = e0;
}
__global__ void k_graph_advance(int32_t* k, uint32_t* epoch, uint32_t inc) {
    *k += 1;
    *epoch += inc;
}

int fill_i32(sf_context* c, int32_t* p, int n, int32_t v) {
    hipLaunchKernelGGL(k_fill_i32, dim3((n + 255) / 256), dim3(256), 0, c->stream, p, n, v);
    return hipGetLastError() == hipSuccess ? SF_OK : SF_ERR_HIP;
}

// Per-chain counters of the cooperative factor, cleared before each launch.
int zero_factor_counters(sf_context* c) { return fill_i32(c, (int32_t*)c->counters, 2 * sfdd::F2_COUNTERS * c->nsub, 0); }

// Pinned staging layout: status word at 0, flags at 64, then three arrays of
// B 8-byte slots (A: done flags / norms, B: relres, C: sweeps).
constexpr size_t STAGE_FLAGS = 64, STAGE_A = 128;
inline char* stage_a(sf_context* c) { return (char*)c->host_stage + STAGE_A; }
inline char* stage_b(sf_context* c) { return stage_a(c) + 8 * (size_t)c->B; }
inline char* stage_c(sf_context* c) { return stage_b(c) + 8 * (size_t)c->B; }
// Convergence-check slots: status, then B done flags, 64-byte aligned.
inline size_t poll_slot_bytes(int B) { return (64 + 4 * (size_t)B + 63) / 64 * 64; }
inline sfdd::DevStatus* poll_status(sf_context* c, int s) {
    return (sfdd::DevStatus*)((char*)c->host_poll + s * poll_slot_bytes(c->B));
}
inline int32_t* poll_done(sf_context* c, int s) { return (int32_t*)((char*)poll_status(c, s) + 64); }
// Queue the copies of the done flags and the status into slot s, then its event.
static int poll_record(sf_context* c, int s) {
    SF_HIP(hipMemcpyAsync(poll_done(c, s), c->done_d, c->B * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipMemcpyAsync(poll_status(c, s), c->status_d, sizeof(sfdd::DevStatus), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipEventRecord(c->poll_ev[s], c->stream));
    return SF_OK;
}
// Wait for slot s; *stop when every pair is done or a device wait was abandoned.
static int poll_check(sf_context* c, int s, bool* stop) {
    SF_HIP(hipEventSynchronize(c->poll_ev[s]));
    bool all = true;
    for (int b = 0; b < c->B; ++b) all = all && poll_done(c, s)[b];
    *stop = all || poll_status(c, s)->code != SF_OK;
    return SF_OK;
}

int pull_status(sf_context* c) {
    sfdd::DevStatus* hs = (sfdd::DevStatus*)c->host_stage;
    SF_HIP(hipMemcpyAsync(hs, c->status_d, sizeof(sfdd::DevStatus), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipStreamSynchronize(c->stream));
    c->status_h = *hs;
    return c->status_h.code;
}

// Tile cuts c_k = floor(k N / P).
int cut(int k, int N, int P) { return (int)(((int64_t)k * N) / P); }

int check_config(const sf_config& k) {
    if (k.width < 2 || k.height < 2 || k.batch < 1) return SF_ERR_INVALID;
    if (k.parts_x < 1 || k.parts_y < 1 || k.parts_x > k.width || k.parts_y > k.height) return SF_ERR_INVALID;
    if (k.overlap < 0 || !(k.lambda > 0.0) || !std::isfinite(k.lambda)) return SF_ERR_INVALID;
    if (!(k.sigma >= 0.0 && k.sigma <= SF_SIGMA_MAX) || !(k.rho >= 0.0 && k.rho <= SF_SIGMA_MAX) ||
        (k.factor_precision != SF_FP64 && k.factor_precision != SF_FP32 && k.factor_precision != SF_FP32_FACTOR) ||
        !(k.pivot_tol >= 0.0 && k.pivot_tol < 1.0) || (k.deferred_status != 0 && k.deferred_status != 1) ||
        k.band_tile < 0)
        return SF_ERR_INVALID;
    if ((int64_t)k.width * k.height * k.batch > (1ll << 31)) return SF_ERR_INVALID;
    return SF_OK;
}

// Subdomains of all pairs, row-major tile order within a pair (Section 3.1):
// tile (p, q) owns [cx_p, cx_{p+1}) x [cy_q, cy_{q+1}); its box grows by
// floor(delta/2) on interior left/top sides and ceil(delta/2) on interior
// right/bottom sides; lines run along the shorter box side.
std::vector<SubDesc> plan_subdomains(const sf_config& k) {
    std::vector<SubDesc> out;
    const int lo = k.overlap / 2, hi = k.overlap - lo;
    for (int pair = 0; pair < k.batch; ++pair)
        for (int q = 0; q < k.parts_y; ++q)
            for (int p = 0; p < k.parts_x; ++p) {
                SubDesc d;
                std::memset(&d, 0, sizeof(d));
                d.pair = pair;
                d.ox0 = cut(p, k.width, k.parts_x);
                d.ox1 = cut(p + 1, k.width, k.parts_x);
                d.oy0 = cut(q, k.height, k.parts_y);
                d.oy1 = cut(q + 1, k.height, k.parts_y);
                const int bx0 = p > 0 ? std::max(0, d.ox0 - lo) : 0;
                const int bx1 = p < k.parts_x - 1 ? std::min(k.width, d.ox1 + hi) : k.width;
                const int by0 = q > 0 ? std::max(0, d.oy0 - lo) : 0;
                const int by1 = q < k.parts_y - 1 ? std::min(k.height, d.oy1 + hi) : k.height;
                d.bx0 = bx0;
                d.by0 = by0;
                d.bw = bx1 - bx0;
                d.bh = by1 - by0;
                d.cols = d.bh <= d.bw;
                d.ms = d.cols ? d.bh : d.bw;
                d.nt = d.cols ? d.bw : d.bh;
                d.m = 3 * d.ms;
                d.NT = (d.m + sfdd::TS - 1) / sfdd::TS;
                d.mp = d.NT * sfdd::TS;
                d.ntiles = d.NT * (d.NT + 1) / 2;
                out.push_back(d);
            }
    return out;
}

}  // namespace

namespace sfdd {

int prof_begin(sf_context* c, int kind) {
    if (!c->profiling) return SF_OK;
    const int need = 2 * (c->ev_used + 1);
    while ((int)c->ev_pool.size() < need) {
        hipEvent_t e;
        SF_HIP(hipEventCreate(&e));
        c->ev_pool.push_back(e);
    }
    c->ev_kind.resize(c->ev_used + 1);
    c->ev_kind[c->ev_used] = kind;
    SF_HIP(hipEventRecord(c->ev_pool[2 * c->ev_used], c->stream));
    return SF_OK;
}

int prof_end(sf_context* c) {
    if (!c->profiling) return SF_OK;
    SF_HIP(hipEventRecord(c->ev_pool[2 * c->ev_used + 1], c->stream));
    ++c->ev_used;
    return SF_OK;
}

int prof_harvest(sf_context* c) {
    if (!c->profiling || c->ev_used == 0) return SF_OK;
    SF_HIP(hipEventSynchronize(c->ev_pool[2 * c->ev_used - 1]));
    for (int i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        SF_HIP(hipEventElapsedTime(&ms, c->ev_pool[2 * i], c->ev_pool[2 * i + 1]));
        c->prof_ms[c->ev_kind[i]] += ms;
        c->prof_n[c->ev_kind[i]] += 1;
    }
    c->ev_used = 0;
    return SF_OK;
}

}  // namespace sfdd

#ifndef SFDD_SOURCE_DIGEST
#define SFDD_SOURCE_DIGEST "unknown"
#endif

extern "C" {

const char* sf_build_digest(void) { return SFDD_SOURCE_DIGEST; }

const char* sf_status_string(int s) {
    switch (s) {
        case SF_OK: return "ok";
        case SF_ERR_INVALID: return "invalid argument";
        case SF_ERR_HIP: return "HIP runtime error";
        case SF_ERR_OOM: return "device out of memory";
        case SF_ERR_STATE: return "call out of order";
        case SF_ERR_DEVICE: return "device-side wait abandoned";
        case SF_NOT_SPD: return "subdomain matrix not positive definite";
        case SF_NOT_CONVERGED: return "not converged within max_sweeps";
        case SF_NONFINITE: return "non-finite value";
        default: return "unknown status";
    }
}

// The graph path's stream, events and device counters (all or none exist).
static void release_graph_resources(sf_context* c) {
    if (c->gk_d) (void)hipFree(c->gk_d);
    if (c->gepoch_d) (void)hipFree(c->gepoch_d);
    for (hipEvent_t& e : c->gev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    c->gk_d = nullptr;
    c->gepoch_d = nullptr;
    c->gstream = nullptr;
}

void sf_destroy(sf_context* c) {
    if (!c) return;
    void* ptrs[] = {c->d_subs, c->f0, c->ft, c->alpha, c->F, c->r, c->eta, c->Fn2, c->Gn2,
                    c->partials, c->relres_d, c->sweeps_d, c->done_d, c->counters, c->etamax_bits,
                    c->flags_d, c->factors, c->work, c->status_d, c->blur_w, c->clg_w, c->coef, c->clg_tmp,
                    c->fail_d, c->sublist_d};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->host_stage) (void)hipHostFree(c->host_stage);
    if (c->host_fail) (void)hipHostFree(c->host_fail);
    if (c->host_poll) (void)hipHostFree(c->host_poll);
    for (hipEvent_t e : c->poll_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    release_graph_resources(c);
    delete c;
}

// Sweep workgroups per chain (P, clamped to the line matrices' block rows and
// to co-residency) and the launch shape that follows; host side only.
// Storage offsets of every subdomain (factors and workspace, in doubles);
// host only.  The totals are the two large device arrays of a context.
static void storage_offsets(std::vector<SubDesc>& subs, int precision, int64_t* factor_doubles,
                            int64_t* work_doubles) {
    int64_t foff = 0, woff = 0, ws = 0;
    for (auto& d : subs) {
        d.foff = foff;
        // tiles in doubles, or in floats packed two per double
        foff += (int64_t)d.nt * d.ntiles * sfdd::TSZ / (precision != SF_FP64 ? 2 : 1);
        d.boff = foff;
        foff += (int64_t)d.nt * d.m * 6;
        d.aoff = foff;
        foff += (int64_t)d.nt * d.ms * 18;
        d.woff = woff;
        woff += (int64_t)d.nt * d.mp;
        d.poff = woff;
        woff += (int64_t)12 * d.mp;
        // factor workspace (one-workgroup factor: 3 mp^2; cooperative: two chains)
        ws = std::max<int64_t>(ws, std::max<int64_t>((int64_t)3 * d.mp * d.mp, 2 * sfdd::f2_chain_doubles(d.mp, d.NT)));
    }
    // The factor runs in chunks of at most FACTOR_WS_SLOTS consecutive
    // subdomains, one chunk after another on the stream, so subdomain i uses
    // workspace slot i mod FACTOR_WS_SLOTS (distinct within any chunk).
    const int nslot = std::min<int>((int)subs.size(), sfdd::FACTOR_WS_SLOTS);
    for (size_t i = 0; i < subs.size(); ++i) subs[i].soff = woff + (int64_t)(i % sfdd::FACTOR_WS_SLOTS) * ws;
    woff += (int64_t)nslot * ws;
    *factor_doubles = foff;
    *work_doubles = woff;
}

// Device bytes of the field arrays of a context (everything but factors and
// workspace), matching the allocations of sf_create.
static int64_t field_bytes(const sf_config& k, int64_t nsub) {
    const int64_t nn = (int64_t)k.width * k.height, ne = (int64_t)(k.width - 1) * (k.height - 1) * 2;
    const int64_t B = k.batch, npart = (nn + 255) / 256;
    int64_t d = 2 * nn * B + 2 * ne * B + 6 * nn * B;          // f0, ft, alpha, eta, F, r
    d += 2 * B + npart * B + B;                                  // Fn2, Gn2, partials, relres
    int64_t bytes = d * 8 + (int64_t)sizeof(SubDesc) * nsub;
    bytes += 4 * (2 * B) + 8 * B + 4 * (2 * sfdd::F2_COUNTERS * nsub) + 16 + sizeof(sfdd::DevStatus);
    bytes += 4 * nsub + 4;                                          // factor failure flags, subdomain list
    if (k.sigma > 0.0) bytes += 8 * (2 * (int64_t)std::ceil(3.0 * k.sigma) + 1);   // blur weights
    if (k.rho > 0.0)                                    // K_rho weights, coefficient planes and first-pass sums
        bytes += 8 * (2 * (int64_t)std::ceil(3.0 * k.rho) + 1) + 2 * 8 * (int64_t)sfdd::CLG_COEFS * ne * B;
    return bytes;
}

// Lanes and chunk of a launch whose subdomains need `per` co-resident
// workgroups each: 8 lanes (a subdomain's workgroups g all have g % 8 equal,
// so they run on one XCD) when 8 subdomains fit, else the largest power of
// two that fits; chunk = the most subdomains, a multiple of the lanes, that
// fit (0 if one does not), at most `cap_chunk` and no more than needed.
static void chunk_shape(int capacity, int per, int nsub, int cap_chunk, int* lanes, int* chunk) {
    int L = 8;
    while (L > 1 && (int64_t)L * per > capacity) L /= 2;
    *lanes = L;
    if (per < 1 || per > capacity) { *chunk = 0; return; }
    const int ch = std::min(L * (capacity / (L * per)), L * (cap_chunk / L));
    *chunk = std::min(ch, L * ((nsub + L - 1) / L));
}

// Shape of a factor or sweep launch, `per` co-resident workgroups per
// subdomain: `main` subdomains side by side in groups of `lanes`
// (chunk_shape), then as many more as the co-resident workgroups left over
// hold, each on `per` contiguous workgroups (its ranks spread over XCDs: the
// exchanges between them are device-scope, so only their latency differs).
// `chunk` is the launch size that needs the fewest launches, balanced.
static void launch_shape(int capacity, int per, int nsub, int cap_chunk, int* lanes, int* main, int* chunk) {
    int ch = 0;
    chunk_shape(capacity, per, nsub, cap_chunk, lanes, &ch);
    const int L = *lanes;
    *main = per >= 1 && per <= capacity ? L * (capacity / (L * per)) : 0;
    if (*main == 0) { *chunk = 0; return; }
    const int tail = (capacity - *main * per) / per;
    const int most = std::max(1, std::min(std::min(*main + tail, cap_chunk), nsub));
    // the fewest launches, balanced: a tail is used only where it saves a launch
    const int launches = (nsub + most - 1) / most;
    *chunk = std::max(1, (nsub + launches - 1) / launches);
}

// Sweep workgroups per chain P and the launch shape that follows (chunks of
// subdomains whose G P ranks each fit co-resident); host side only.
static void set_sweep_shape(sf_context* c, int P) {
    int maxnt = 0;
    for (const auto& d : c->subs) maxnt = std::max(maxnt, d.NT);
    const int G = c->groups;
    // ranks beyond a subdomain's block rows have nothing to do
    P = std::max(1, std::min(std::min(P, maxnt), 255));
    if (G * P > c->sweep_capacity) P = std::max(1, c->sweep_capacity / G);
    c->maxP = P;
    launch_shape(c->sweep_capacity, G * P, c->nsub, 1 << 30, &c->sweep_lanes, &c->sweep_main, &c->sweep_chunk);
    c->sweep_rows = 0;
    for (int r = 0; r < P; ++r) {
        int R = 0;
        while (2 * P * (R / 2) + ((R & 1) ? 2 * P - 1 - r : r) < maxnt) ++R;
        c->sweep_rows = std::max(c->sweep_rows, R);
    }
    for (auto& d : c->subs) d.P = P;
}

int sf_create(const sf_config* cfg, void* stream, sf_context** out) {
    if (!cfg || !out) return SF_ERR_INVALID;
    *out = nullptr;
    const sf_config k = *cfg;
    SF_TRY(check_config(k));

    sf_context* c = new (std::nothrow) sf_context();   // value-initialised: null pointers
    if (!c) return SF_ERR_OOM;
    c->cfg = k;
    c->stream = (hipStream_t)stream;
    c->W = k.width;
    c->H = k.height;
    c->B = k.batch;
    c->wait_limit = 1ll << 20;
    if (hipGetDevice(&c->device) != hipSuccess) { sf_destroy(c); return SF_ERR_HIP; }
    // the allocation-free entry point's static array: its address on this
    // device (looked up once per device, with the device current)
    {
        const int rc = sfdd::scratch_resolve(c->device, &c->scratch);
        if (rc != SF_OK) { sf_destroy(c); return rc; }
    }

    // ---- geometry (Section 3.1) --------------------------------------------
    c->subs = plan_subdomains(k);
    int maxmp = 0, maxnt = 0;
    for (const auto& d : c->subs) {
        maxmp = std::max(maxmp, d.mp);
        maxnt = std::max(maxnt, d.NT);
    }
    if (maxmp > MAX_LINE) { sf_destroy(c); return SF_ERR_INVALID; }   // line matrices up to 768 x 768
    c->nsub = (int)c->subs.size();

    // ---- launch shapes ---------------------------------------------------------
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        sf_destroy(c);
        return SF_ERR_HIP;
    }
    // co-resident sweep workgroups: the least of the forms this precision uses
    int occ = 1 << 30;
    const int fp32 = k.factor_precision != SF_FP64;
    for (int form : {sfdd::SWEEP_GENERAL, sfdd::SWEEP_FAST2, sfdd::SWEEP_FAST1}) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sfdd::sweep_kernel(form, fp32), sfdd::sweep_threads(form),
                                                         0) != hipSuccess || o < 1)
            o = 1;
        occ = std::min(occ, o);
    }
    const int capacity = ncu * occ;
    c->sweep_capacity = capacity;

    // cooperative factor: f2_ranks(NT) workgroups and a pivot server per
    // chain, line matrices up to 768; two chains per subdomain (twisted
    // factorisation) when 8 subdomains fit one launch with both chains in the
    // factor and with the fast sweep's ranks, else one chain
    int occ2 = 0;
    // (both arithmetic forms of the cooperative factor: the least of the two)
    for (int f32 = 0; f32 < 2; ++f32) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sfdd::factor2_kernel(f32), sfdd::F2_WAVES * 64, 0) !=
            hipSuccess)
            o = 0;
        occ2 = f32 == 0 ? o : std::min(occ2, o);
    }
    const int fcap = ncu * occ2;
    int Pf = 0;
    for (const auto& d : c->subs) Pf = std::max(Pf, sfdd::f2_ranks(d.NT));
    const int Pfast = maxnt <= 14 ? (maxnt + 1) / 2 : maxnt;   // fast sweep: 2 block rows per rank, or 1
    c->groups = 1;
    if (maxnt <= sfdd::F2_MAX_NT && occ2 >= 1 && Pf + 1 <= fcap) {
        c->factor_pf = Pf;
        if (8 * 2 * (Pf + 1) <= fcap && 8 * 2 * Pfast <= capacity) c->groups = 2;
        launch_shape(fcap, c->groups * (Pf + 1), c->nsub, sfdd::FACTOR_WS_SLOTS, &c->factor_lanes, &c->factor_main,
                     &c->factor_chunk);
    } else {
        // one workgroup per subdomain (line matrices up to 512)
        if (maxmp > 512) { sf_destroy(c); return SF_ERR_INVALID; }
        c->factor_pf = 0;
        c->factor_lanes = 1;
        c->factor_main = 1;
        c->factor_chunk = std::min(c->nsub, sfdd::FACTOR_WS_SLOTS);
    }
    const int G = c->groups;

    // sweep workgroups per chain: the fast forms' count, or more where that
    // keeps a fast form (lines up to 14 block rows; some ranks then own one
    // block row and others two) and needs no more launches per sweep
    int P;
    if (k.band_tile > 0) {
        P = k.band_tile;
    } else {
        auto launches = [&](int p) {
            int L = 0, m = 0, ch = 0;
            launch_shape(capacity, G * p, c->nsub, 1 << 30, &L, &m, &ch);
            return ch > 0 ? (c->nsub + ch - 1) / ch : c->nsub + 1;
        };
        P = Pfast;
        if (maxnt <= 14) {
            const int n0 = launches(Pfast);
            for (int p = maxnt; p > Pfast; --p)
                if (G * p <= capacity && launches(p) <= n0) {
                    P = p;
                    break;
                }
        }
    }
    set_sweep_shape(c, P);

    // ---- storage offsets -----------------------------------------------------
    for (auto& d : c->subs) d.kmid = G == 2 ? (d.nt - 1) / 2 : d.nt - 1;
    storage_offsets(c->subs, k.factor_precision, &c->factor_doubles, &c->work_doubles);

    const int64_t nn = (int64_t)c->W * c->H, ne = (int64_t)(c->W - 1) * (c->H - 1) * 2;
    c->npart = (int)((nn + 255) / 256);
    int rc = SF_OK;
    rc |= dalloc(&c->d_subs, c->subs.size());
    rc |= dalloc(&c->f0, nn * c->B);
    rc |= dalloc(&c->ft, nn * c->B);
    rc |= dalloc(&c->alpha, ne * c->B);
    rc |= dalloc(&c->eta, ne * c->B);
    rc |= dalloc(&c->F, 3 * nn * c->B);
    rc |= dalloc(&c->r, 3 * nn * c->B);
    rc |= dalloc(&c->Fn2, c->B);
    rc |= dalloc(&c->Gn2, c->B);
    rc |= dalloc(&c->partials, (size_t)c->npart * c->B);
    rc |= dalloc(&c->relres_d, c->B);
    rc |= dalloc(&c->sweeps_d, c->B);
    rc |= dalloc(&c->done_d, c->B);
    rc |= dalloc(&c->counters, 2 * sfdd::F2_COUNTERS * (size_t)c->nsub);
    rc |= dalloc(&c->etamax_bits, c->B);
    rc |= dalloc(&c->flags_d, 4);
    rc |= dalloc(&c->fail_d, c->nsub);
    rc |= dalloc(&c->sublist_d, 1);
    rc |= dalloc(&c->factors, (size_t)c->factor_doubles);
    rc |= dalloc(&c->work, (size_t)c->work_doubles);
    rc |= dalloc(&c->status_d, 1);
    // presmoothing weights K_sigma and data-term weights K_rho (Section 1):
    // sampled Gaussian, |k| <= ceil(3 s), normalised
    auto gauss = [](double sg, int* r) {
        std::vector<double> w;
        *r = (int)std::ceil(3.0 * sg);
        double sum = 0.0;
        for (int i = -*r; i <= *r; ++i) {
            w.push_back(std::exp(-(double)i * i / (2.0 * sg * sg)));
            sum += w.back();
        }
        for (auto& v : w) v /= sum;
        return w;
    };
    std::vector<double> bw, cw;
    if (k.sigma > 0.0) {
        bw = gauss(k.sigma, &c->blur_r);
        rc |= dalloc(&c->blur_w, bw.size());
    }
    if (k.rho > 0.0) {
        cw = gauss(k.rho, &c->clg_r);
        rc |= dalloc(&c->clg_w, cw.size());
        rc |= dalloc(&c->coef, (size_t)sfdd::CLG_COEFS * ne * c->B);
        rc |= dalloc(&c->clg_tmp, (size_t)sfdd::CLG_COEFS * ne * c->B);
    }
    if (rc != SF_OK) { sf_destroy(c); return SF_ERR_OOM; }
    const size_t stage = STAGE_A + 24 * (size_t)c->B + 64;
    if (hipHostMalloc(&c->host_stage, stage, hipHostMallocDefault) != hipSuccess) {
        c->host_stage = nullptr;
        sf_destroy(c);
        return SF_ERR_OOM;
    }
    if (hipHostMalloc(&c->host_fail, sizeof(int32_t) * (size_t)c->nsub, hipHostMallocDefault) != hipSuccess) {
        c->host_fail = nullptr;
        sf_destroy(c);
        return SF_ERR_OOM;
    }
    if (hipHostMalloc(&c->host_poll, 2 * poll_slot_bytes(c->B), hipHostMallocDefault) != hipSuccess) {
        c->host_poll = nullptr;
        sf_destroy(c);
        return SF_ERR_OOM;
    }
    for (hipEvent_t& e : c->poll_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
            sf_destroy(c);
            return SF_ERR_HIP;
        }
    // uploads and clears go on the context's stream, so the synchronisation
    // below covers them also when that stream does not wait for the null stream
    if (hipMemcpyAsync(c->d_subs, c->subs.data(), c->subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess) {
        sf_destroy(c);
        return SF_ERR_HIP;
    }
    // sweep exchange buffers start with tag 0, which no launch ever waits for
    if (hipMemsetAsync(c->work, 0, (size_t)c->work_doubles * sizeof(double), c->stream) != hipSuccess) {
        sf_destroy(c);
        return SF_ERR_HIP;
    }
    c->sweep_epoch = 1;
    c->factor_epoch = 1;
    if ((!bw.empty() &&
         hipMemcpyAsync(c->blur_w, bw.data(), bw.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) !=
             hipSuccess) ||
        (!cw.empty() &&
         hipMemcpyAsync(c->clg_w, cw.data(), cw.size() * sizeof(double), hipMemcpyHostToDevice, c->stream) !=
             hipSuccess)) {
        sf_destroy(c);
        return SF_ERR_HIP;
    }

    hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        sf_destroy(c);
        return SF_ERR_HIP;
    }
    c->state = ST_CREATED;
    *out = c;
    return SF_OK;
}

// The input check of sf_assemble: the flags k_validate left (waits for the stream).
static int assemble_status(sf_context* c) {
    int32_t* hf = (int32_t*)((char*)c->host_stage + STAGE_FLAGS);
    SF_HIP(hipMemcpyAsync(hf, c->flags_d, 4 * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipStreamSynchronize(c->stream));
    if (hf[0] || hf[1]) return hf[0] ? SF_NONFINITE : SF_ERR_INVALID;
    return SF_OK;
}

int sf_assemble(sf_context* c, const double* I0, const double* I1, const double* alpha) {
    if (!c || !I0 || !I1 || !alpha) return SF_ERR_INVALID;
    c->state = ST_CREATED;
    c->pending = 0;                         // a status of earlier data no longer applies
    SF_TRY(sfdd::prof_begin(c, sfdd::PROF_OTHER));
    SF_TRY(fill_i32(c, c->flags_d, 4, 0));
    SF_TRY(sfdd::launch_validate(c, I0, I1, alpha));
    if (c->cfg.deferred_status) {
        // the kernels below run on whatever the frames hold; the check is
        // reported by the next call that collects the status
        c->pending |= PENDING_ASSEMBLE;
    } else {
        const int code = assemble_status(c);
        if (code != SF_OK) {
            SF_TRY(sfdd::prof_end(c));
            return code;
        }
    }
    if (c->blur_r > 0) {
        // smoothed frames in the residual array (free until the first solve)
        const int64_t n = (int64_t)c->W * c->H * c->B;
        double* s0 = c->r;
        double* s1 = c->r + n;
        double* tmp = c->r + 2 * n;
        SF_TRY(sfdd::launch_presmooth(c, I0, s0, tmp));
        SF_TRY(sfdd::launch_presmooth(c, I1, s1, tmp));
        SF_TRY(sfdd::launch_assemble(c, s0, s1, alpha));
    } else {
        SF_TRY(sfdd::launch_assemble(c, I0, I1, alpha));
    }
    // K_rho data term: coefficient planes from the (smoothed) frames, then F
    if (c->coef) SF_TRY(sfdd::launch_clg(c));
    SF_TRY(sfdd::prof_end(c));
    c->state = ST_ASSEMBLED;
    return SF_OK;
}

// Sweeps and factorisations of different contexts do not run at the same
// time on one device: a sweep or factor launch may take the device's whole
// co-resident capacity and its workgroups wait on each other, so two
// overlapping launches could each hold part of the device while waiting for
// workgroups that cannot become resident (until the wait bound ends them
// with SF_ERR_DEVICE).  Every call that launches them (and waits for them)
// holds its device's lock until its streams have drained; within one process
// such calls therefore run one at a time per device.  Recursive: the FP64
// refactorisation inside a factorisation's status collection takes it again.
static std::recursive_mutex& sweep_mutex(int device) {
    static std::recursive_mutex m[64];
    return m[device & 63];
}
struct SweepLock {
    sf_context* c;
    explicit SweepLock(sf_context* ctx) : c(ctx) { sweep_mutex(c->device).lock(); }
    ~SweepLock() {
        (void)hipStreamSynchronize(c->stream);
        if (c->gstream) (void)hipStreamSynchronize(c->gstream);
        sweep_mutex(c->device).unlock();
    }
    SweepLock(const SweepLock&) = delete;
    SweepLock& operator=(const SweepLock&) = delete;
};

static int factor_status(sf_context* c);

int sf_factor_subdomains(sf_context* c) {
    if (!c) return SF_ERR_INVALID;
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    // waiting for the status: the launches are serialised with other contexts'
    // (with deferred status the call only enqueues and takes no lock)
    std::optional<SweepLock> lock;
    if (!c->cfg.deferred_status) lock.emplace(c);
    c->state = ST_ASSEMBLED;                // until the new factors are complete
    SF_TRY(sfdd::prof_begin(c, sfdd::PROF_FACTOR));
    const int fp32_arith = c->cfg.factor_precision == SF_FP32_FACTOR && c->factor_pf > 0;
    c->pending &= ~PENDING_FACTOR;
    if (c->factor_pf > 0) {
        SF_TRY(sfdd::launch_line_coeffs(c));
        hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
        SF_HIP(hipGetLastError());
        if (fp32_arith) SF_TRY(fill_i32(c, c->fail_d, c->nsub, 0));
        // a pivot of the FP32 factorisation is rejected below pivot_tol (its
        // subdomain is then factored again in FP64), one of the FP64
        // factorisation below 1e-13 (SF_NOT_SPD)
        const double ptol = fp32_arith ? (c->cfg.pivot_tol > 0.0 ? c->cfg.pivot_tol : 1e-5) : 1e-13;
        for (int s0 = 0; s0 < c->nsub; s0 += c->factor_chunk) {
            const int n = std::min(c->factor_chunk, c->nsub - s0);
            SF_TRY(zero_factor_counters(c));
            SF_TRY(sfdd::launch_factor2(c, s0, n, c->factor_pf, fp32_arith, nullptr, c->factor_lanes, c->factor_main,
                                        ptol));
        }
    } else {
        SF_TRY(sfdd::launch_factor(c));
    }
    SF_TRY(sfdd::prof_end(c));
    c->state = ST_FACTORED;
    if (c->cfg.deferred_status) {
        c->pending |= PENDING_FACTOR;
        return SF_OK;
    }
    return factor_status(c);
}

// The pivot status of the factorisation just enqueued (waits for the
// stream); with FP32 arithmetic, subdomains with a rejected pivot are
// factored again in FP64 here.  On an error the factors are unusable.
static int factor_status(sf_context* c) {
    const int fp32_arith = c->cfg.factor_precision == SF_FP32_FACTOR && c->factor_pf > 0;
    int code = pull_status(c);
    SF_TRY(sfdd::prof_harvest(c));
    if (fp32_arith && code == SF_NOT_SPD) {
        // FP64 fallback, subdomain by subdomain (each one alone in its launch,
        // so the factor workspace slots cannot collide)
        SweepLock lock(c);
        int32_t* hf = (int32_t*)c->host_fail;
        SF_HIP(hipMemcpyAsync(hf, c->fail_d, c->nsub * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        SF_HIP(hipStreamSynchronize(c->stream));
        hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
        SF_HIP(hipGetLastError());
        c->fp64_fallbacks = 0;
        SF_TRY(sfdd::prof_begin(c, sfdd::PROF_FACTOR));
        for (int i = 0; i < c->nsub; ++i) {
            if (!hf[i]) continue;
            ++c->fp64_fallbacks;
            hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(1), 0, c->stream, c->sublist_d, 1, (int32_t)i);
            SF_HIP(hipGetLastError());
            SF_TRY(zero_factor_counters(c));
            SF_TRY(sfdd::launch_factor2(c, 0, 1, sfdd::f2_ranks(c->subs[i].NT), 0, c->sublist_d, 1, 1, 1e-13));
        }
        SF_TRY(sfdd::prof_end(c));
        code = pull_status(c);
        SF_TRY(sfdd::prof_harvest(c));
    } else {
        c->fp64_fallbacks = 0;
    }
    if (code != SF_OK) {
        c->state = ST_ASSEMBLED;
        return code;
    }
    return SF_OK;
}

#define SF_SETTLE(c)                           \
    do {                                       \
        const int sc_ = settle(c);             \
        if (sc_ != SF_OK) return sc_;          \
    } while (0)

// Collect what sf_assemble / sf_factor_subdomains left pending (deferred
// status): the input check first (on an error the context is back to
// created), then the pivot status.
static int settle(sf_context* c) {
    if (c->pending & PENDING_ASSEMBLE) {
        c->pending &= ~PENDING_ASSEMBLE;
        const int code = assemble_status(c);
        if (code != SF_OK) {
            c->pending = 0;
            c->state = ST_CREATED;
            return code;
        }
    }
    if (c->pending & PENDING_FACTOR) {
        c->pending &= ~PENDING_FACTOR;
        return factor_status(c);
    }
    return SF_OK;
}

int sf_sync(sf_context* c) {
    if (!c) return SF_ERR_INVALID;
    const int code = settle(c);
    if (code != SF_OK) return code;
    SF_HIP(hipStreamSynchronize(c->stream));
    return SF_OK;
}

int sf_set_wait_limit(sf_context* c, int64_t polls) {
    if (!c || polls < 0) return SF_ERR_INVALID;
    c->wait_limit = (long long)polls;
    return SF_OK;
}

// RAS iteration on A U = rhs from the U given, stopping per pair at
// ||rhs - A U|| <= rtol ||rhs|| (rhs_n2 = ||rhs||^2 on the device).
// Prologue: pairs with rhs = 0 get U = 0; all pairs active; status cleared.
static int loop_prologue(sf_context* c, double* U, const double* rhs_n2) {
    SF_TRY(sfdd::prof_begin(c, sfdd::PROF_OTHER));
    SF_TRY(sfdd::launch_zero_where_rhs_zero(c, U, rhs_n2));
    SF_TRY(fill_i32(c, c->done_d, c->B, 0));
    hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
    SF_HIP(hipGetLastError());
    return sfdd::prof_end(c);
}

// Iterations k0 .. max_sweeps, one launch each (residual + convergence test,
// then a sweep).  Every 4 sweeps the done flags and the status are copied to
// a host slot behind an event; the host reads the previous check while the
// next 4 iterations are already queued, so the device never waits for the
// host.  A pair that is done makes every kernel of the pair return at once,
// so the iterations queued past convergence cost their launches only.
static int loop_iterations(sf_context* c, double* U, const double* rhs, const double* rhs_n2, double rtol,
                           int32_t max_sweeps, int k0) {
    const int check_every = 4;
    int nchk = 0;
    for (int k = k0; k <= max_sweeps; ++k) {
        SF_TRY(sfdd::prof_begin(c, sfdd::PROF_RESIDUAL));
        SF_TRY(sfdd::launch_residual(c, U, c->r, 1, rtol, k, max_sweeps, rhs, rhs_n2));
        SF_TRY(sfdd::prof_end(c));
        if (k == max_sweeps) break;
        SF_TRY(sfdd::prof_begin(c, sfdd::PROF_SWEEP));
        SF_TRY(sfdd::launch_sweep(c, U, c->r, -1, nullptr, nullptr));
        SF_TRY(sfdd::prof_end(c));
        if ((k + 1) % check_every == 0) {
            SF_TRY(poll_record(c, nchk & 1));
            ++nchk;
            if (nchk >= 2) {
                bool stop = false;
                SF_TRY(poll_check(c, (nchk - 2) & 1, &stop));
                if (stop) break;
            }
        }
    }
    return SF_OK;
}

// Per-pair results of the loop and its status.
static int loop_finish(sf_context* c, double rtol, int32_t* sweeps, double* relres) {
    double* hrel = (double*)stage_b(c);
    int32_t* hsw = (int32_t*)stage_c(c);
    SF_HIP(hipMemcpyAsync(hrel, c->relres_d, c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipMemcpyAsync(hsw, c->sweeps_d, c->B * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    SF_HIP(hipStreamSynchronize(c->stream));
    SF_TRY(sfdd::prof_harvest(c));
    int rc = SF_OK;
    for (int b = 0; b < c->B; ++b) {
        if (relres) relres[b] = hrel[b];
        if (sweeps) sweeps[b] = hsw[b];
        if (!std::isfinite(hrel[b])) rc = SF_NONFINITE;
        else if (hrel[b] > rtol && rc == SF_OK) rc = SF_NOT_CONVERGED;
    }
    const int code = pull_status(c);
    if (code != SF_OK) return code;
    return rc;
}

static int schwarz_loop(sf_context* c, double* U, const double* rhs, const double* rhs_n2, double rtol,
                        int32_t max_sweeps, int32_t* sweeps, double* relres) {
    SF_TRY(loop_prologue(c, U, rhs_n2));
    SF_TRY(loop_iterations(c, U, rhs, rhs_n2, rtol, max_sweeps, 0));
    return loop_finish(c, rtol, sweeps, relres);
}

// Graph-replayed iterations on c->stream (the private stream): one chunk of
// GRAPH_CHUNK iterations (residual + convergence test, sweep, advance of the
// device counters) and the copies of the done flags and status is captured
// once and replayed while whole chunks fit in max_sweeps and some pair is
// active.  *k_next: the first iteration not run (max_sweeps + 1 when every
// pair finished or a device wait was abandoned).
constexpr int GRAPH_CHUNK = 4;
static int graph_iterations(sf_context* c, double* U, double rtol, int32_t max_sweeps, int* k_next) {
    *k_next = 0;
    if (max_sweeps < GRAPH_CHUNK) return SF_OK;
    const uint32_t e0 = c->sweep_epoch, inc = sfdd::sweep_epoch_step(c);
    hipLaunchKernelGGL(k_graph_init, dim3(1), dim3(1), 0, c->stream, c->gk_d, c->gepoch_d, e0);
    SF_HIP(hipGetLastError());
    int32_t* hd = (int32_t*)stage_a(c);
    sfdd::DevStatus* hst = (sfdd::DevStatus*)c->host_stage;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    SF_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->graph_capture = 1;
    int rc = SF_OK;
    for (int i = 0; i < GRAPH_CHUNK && rc == SF_OK; ++i) {
        rc = sfdd::launch_residual(c, U, c->r, 1, rtol, 0, max_sweeps, c->F, c->Fn2);
        if (rc == SF_OK) rc = sfdd::launch_sweep(c, U, c->r, -1, nullptr, nullptr);
        if (rc == SF_OK) {
            hipLaunchKernelGGL(k_graph_advance, dim3(1), dim3(1), 0, c->stream, c->gk_d, c->gepoch_d, inc);
            if (hipGetLastError() != hipSuccess) rc = SF_ERR_HIP;
        }
    }
    if (rc == SF_OK &&
        hipMemcpyAsync(hd, c->done_d, c->B * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        rc = SF_ERR_HIP;
    if (rc == SF_OK &&
        hipMemcpyAsync(hst, c->status_d, sizeof(sfdd::DevStatus), hipMemcpyDeviceToHost, c->stream) != hipSuccess)
        rc = SF_ERR_HIP;
    c->graph_capture = 0;
    if (hipStreamEndCapture(c->stream, &g) != hipSuccess && rc == SF_OK) rc = SF_ERR_HIP;
    if (rc == SF_OK && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) rc = SF_ERR_HIP;
    // Replays are queued one ahead: after queueing replay r the host waits
    // for replay r - 1 only.  The flags it then reads were copied by replay
    // r - 1 or, already, by replay r: done flags and the status only ever
    // change towards "stop", so either is a valid check.
    int k = 0, replays = 0;
    while (rc == SF_OK && k + GRAPH_CHUNK <= max_sweeps) {
        if (hipGraphLaunch(ge, c->stream) != hipSuccess ||
            hipEventRecord(c->poll_ev[replays & 1], c->stream) != hipSuccess) {
            rc = SF_ERR_HIP;
            break;
        }
        ++replays;
        k += GRAPH_CHUNK;
        if (replays < 2) continue;
        if (hipEventSynchronize(c->poll_ev[(replays - 2) & 1]) != hipSuccess) {
            rc = SF_ERR_HIP;
            break;
        }
        bool all = true;
        for (int b = 0; b < c->B; ++b) all = all && hd[b];
        if (hst->code != SF_OK || all) {
            k = max_sweeps + 1;
            break;
        }
    }
    // the last replays have not been looked at: one more check once they end
    if (rc == SF_OK && k <= max_sweeps && replays > 0) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) {
            rc = SF_ERR_HIP;
        } else {
            bool all = true;
            for (int b = 0; b < c->B; ++b) all = all && hd[b];
            if (hst->code != SF_OK || all) k = max_sweeps + 1;
        }
    }
    // the replays used tag bases e0 .. e0 + (GRAPH_CHUNK replays - 1) inc
    c->sweep_epoch = std::max(c->sweep_epoch, e0 + (uint32_t)(GRAPH_CHUNK * replays) * inc);
    // (a replay may still be running: the executable graph goes once it ends)
    if (replays > 0 && hipStreamSynchronize(c->stream) != hipSuccess && rc == SF_OK) rc = SF_ERR_HIP;
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    *k_next = k;
    return rc;
}

int sf_schwarz_solve_graph(sf_context* c, double* U, double rtol, int32_t max_sweeps, int32_t* sweeps,
                           double* relres) {
    if (!c || !U || max_sweeps < 0 || !(rtol >= 0.0)) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state != ST_FACTORED) return SF_ERR_STATE;
    SweepLock lock(c);
    if (!c->gstream) {
        // created together on first use; a failure leaves none of them, so a
        // later call never runs with a missing counter
        int rc = SF_OK;
        if (hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking) != hipSuccess) {
            c->gstream = nullptr;
            rc = SF_ERR_HIP;
        }
        for (hipEvent_t& e : c->gev)
            if (rc == SF_OK && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                e = nullptr;
                rc = SF_ERR_HIP;
            }
        if (rc == SF_OK) rc = dalloc(&c->gk_d, 1);
        if (rc == SF_OK) rc = dalloc(&c->gepoch_d, 1);
        if (rc != SF_OK) {
            (void)hipGetLastError();
            release_graph_resources(c);
            return rc;
        }
    }
    SF_TRY(loop_prologue(c, U, c->Fn2));
    // the private stream continues after the work queued on the context's stream
    SF_HIP(hipEventRecord(c->gev[0], c->stream));
    SF_HIP(hipStreamWaitEvent(c->gstream, c->gev[0], 0));
    hipStream_t user = c->stream;
    c->stream = c->gstream;
    int k = 0;
    int rc = graph_iterations(c, U, rtol, max_sweeps, &k);
    if (rc == SF_OK && k <= max_sweeps) rc = loop_iterations(c, U, c->F, c->Fn2, rtol, max_sweeps, k);
    c->stream = user;
    // and the context's stream continues after the private one
    if (hipEventRecord(c->gev[1], c->gstream) != hipSuccess || hipStreamWaitEvent(user, c->gev[1], 0) != hipSuccess)
        return SF_ERR_HIP;
    if (rc != SF_OK) return rc;
    return loop_finish(c, rtol, sweeps, relres);
}

int sf_schwarz_solve(sf_context* c, double* U, double rtol, int32_t max_sweeps, int32_t* sweeps, double* relres) {
    if (!c || !U || max_sweeps < 0 || !(rtol >= 0.0)) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state != ST_FACTORED) return SF_ERR_STATE;
    SweepLock lock(c);
    return schwarz_loop(c, U, c->F, c->Fn2, rtol, max_sweeps, sweeps, relres);
}

int sf_autotune(sf_context* c, double* U, int32_t trials, int32_t* band_tile) {
    if (!c || !U || trials < 1) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state != ST_FACTORED) return SF_ERR_STATE;
    SweepLock lock(c);
    int maxnt = 0;
    for (const auto& d : c->subs) maxnt = std::max(maxnt, d.NT);
    // candidates: for every number of block rows per workgroup, the fewest
    // workgroups per chain that give it
    std::vector<int> cand;
    for (int rows = 1; rows <= maxnt; ++rows) {
        const int P = (maxnt + rows - 1) / rows;
        if (cand.empty() || cand.back() != P) cand.push_back(P);
    }
    hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
    SF_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    SF_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SF_ERR_HIP;
    }
    const int keep = c->maxP;
    int best = keep, rc = SF_OK;
    float best_ms = 0.0f;
    std::vector<int> tried;
    for (int P : cand) {
        set_sweep_shape(c, P);
        if (std::find(tried.begin(), tried.end(), c->maxP) != tried.end()) continue;   // clamped to a tried shape
        tried.push_back(c->maxP);
        if (hipMemcpyAsync(c->d_subs, c->subs.data(), c->subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice,
                           c->stream) != hipSuccess) { rc = SF_ERR_HIP; break; }
        if ((rc = fill_i32(c, c->done_d, c->B, 0)) != SF_OK) break;
        if ((rc = sfdd::launch_residual(c, U, c->r, 0, 0.0, 0, 0)) != SF_OK) break;
        if ((rc = sfdd::launch_sweep(c, U, c->r, -1, nullptr, nullptr)) != SF_OK) break;   // warm-up
        if (hipEventRecord(e0, c->stream) != hipSuccess) { rc = SF_ERR_HIP; break; }
        for (int i = 0; i < trials && rc == SF_OK; ++i) rc = sfdd::launch_sweep(c, U, c->r, -1, nullptr, nullptr);
        if (rc != SF_OK) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, c->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) { rc = SF_ERR_HIP; break; }
        const int code = pull_status(c);
        if (code != SF_OK) { rc = code; break; }
        if (tried.size() == 1 || ms < best_ms) {
            best_ms = ms;
            best = c->maxP;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_sweep_shape(c, rc == SF_OK ? best : keep);
    // on the context's stream, after any sweep still queued there (an early
    // break leaves some), so no sweep reads the descriptors while they change
    if (hipMemcpyAsync(c->d_subs, c->subs.data(), c->subs.size() * sizeof(SubDesc), hipMemcpyHostToDevice,
                       c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        return SF_ERR_HIP;
    if (band_tile) *band_tile = c->maxP;
    return rc;
}

int sf_adjoint(sf_context* c, const double* U, const double* G, double* P, double* dI0, double* dI1, double* dalpha,
               double rtol, int32_t max_sweeps, int32_t* sweeps, double* relres) {
    if (!c || !U || !G || !P || max_sweeps < 0 || !(rtol >= 0.0)) return SF_ERR_INVALID;
    // gradients are taken with respect to unsmoothed frames and the plain data term
    if (c->blur_r > 0 || c->coef) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state != ST_FACTORED) return SF_ERR_STATE;
    SweepLock lock(c);
    SF_TRY(sfdd::launch_norm2(c, G, c->Gn2));
    const int rc = schwarz_loop(c, P, G, c->Gn2, rtol, max_sweeps, sweeps, relres);
    if (rc != SF_OK && rc != SF_NOT_CONVERGED) return rc;
    SF_TRY(sfdd::prof_begin(c, sfdd::PROF_OTHER));
    SF_TRY(sfdd::launch_adjoint_gradients(c, U, P, dI0, dI1, dalpha));
    SF_TRY(sfdd::prof_end(c));
    SF_HIP(hipStreamSynchronize(c->stream));
    SF_TRY(sfdd::prof_harvest(c));
    return rc;
}

int sf_update_alpha(sf_context* c, const double* U, double* alpha, double kappa, double eta_thr, double alpha_th,
                    double* eta_max) {
    if (!c || !U || !alpha || !(kappa >= 0.0) || !std::isfinite(eta_thr) || !(alpha_th > 0.0)) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    SF_TRY(sfdd::prof_begin(c, sfdd::PROF_OTHER));
    SF_TRY(sfdd::launch_indicator(c, U, c->eta, 1));
    SF_TRY(sfdd::launch_alpha_update(c, c->eta, alpha, kappa, eta_thr, alpha_th));
    SF_TRY(sfdd::prof_end(c));
    c->state = ST_ASSEMBLED;   // factors are stale, F is unchanged
    if (eta_max) {
        uint64_t* hb = (uint64_t*)stage_a(c);
        SF_HIP(hipMemcpyAsync(hb, c->etamax_bits, c->B * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
        SF_HIP(hipStreamSynchronize(c->stream));
        for (int b = 0; b < c->B; ++b) std::memcpy(&eta_max[b], &hb[b], sizeof(double));
    }
    return SF_OK;
}

int sf_error_detail(const sf_context* c, int32_t* pair, int32_t* subdomain, int64_t* row) {
    if (!c) return SF_ERR_INVALID;
    const int s = c->status_h.sub;
    const int per = c->cfg.parts_x * c->cfg.parts_y;
    if (pair) *pair = s >= 0 ? s / per : -1;
    if (subdomain) *subdomain = s >= 0 ? s % per : -1;
    if (row) *row = c->status_h.row;
    return c->status_h.code;
}

int sf_rhs(sf_context* c, double* F) {
    if (!c || !F) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    SF_HIP(hipMemcpyAsync(F, c->F, 3 * sizeof(double) * c->W * c->H * c->B, hipMemcpyDeviceToDevice, c->stream));
    return SF_OK;
}

int sf_residual(sf_context* c, const double* U, double* r, double* rnorm2) {
    if (!c || !U || !r) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    SF_TRY(sfdd::launch_residual(c, U, r, 0, 0.0, 0, 0));
    if (rnorm2) {
        double* h = (double*)stage_a(c);
        SF_HIP(hipMemcpyAsync(h, c->relres_d, c->B * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        SF_HIP(hipStreamSynchronize(c->stream));
        for (int b = 0; b < c->B; ++b) rnorm2[b] = h[b];
    }
    return SF_OK;
}

int sf_residual_noalloc(sf_context* c, const double* U, double* r, double* rnorm2) {
    if (!c || !U || !r) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    if (!c->scratch) return SF_ERR_STATE;
    if (sfdd::scratch_residual_doubles(c) * (int64_t)sizeof(double) > (int64_t)SF_NOALLOC_SCRATCH_BYTES)
        return SF_ERR_INVALID;   // B * ceil(W H / 256) + B doubles exceed the static array
    SF_TRY(sfdd::launch_residual_scratch(c, U, r, c->scratch));
    if (rnorm2) {
        double* h = (double*)stage_a(c);
        SF_HIP(hipMemcpyAsync(h, c->scratch + (int64_t)c->B * c->npart, c->B * sizeof(double),
                              hipMemcpyDeviceToHost, c->stream));
        SF_HIP(hipStreamSynchronize(c->stream));
        for (int b = 0; b < c->B; ++b) rnorm2[b] = h[b];
    }
    return SF_OK;
}

int sf_indicator(sf_context* c, const double* U, double* eta) {
    if (!c || !U || !eta) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state < ST_ASSEMBLED) return SF_ERR_STATE;
    return sfdd::launch_indicator(c, U, eta, 1);
}

int sf_choose_split(int32_t width, int32_t height, int32_t nparts, int32_t* parts_x, int32_t* parts_y,
                    double* ratio) {
    if (width < 2 || height < 2 || nparts < 1) return SF_ERR_INVALID;
    int bx = 0, by = 0;
    double br = -1.0;
    for (int px = 1; px <= nparts; ++px) {
        if (nparts % px) continue;
        const int py = nparts / px;
        if (px > width || py > height) continue;
        const double w = (double)width / px, h = (double)height / py;
        const double r = (w * h) / (2.0 * (w + h));
        if (r > br || (r == br && px > bx)) {
            bx = px;
            by = py;
            br = r;
        }
    }
    if (bx == 0) return SF_ERR_INVALID;
    if (parts_x) *parts_x = bx;
    if (parts_y) *parts_y = by;
    if (ratio) *ratio = br;
    return SF_OK;
}

int sf_num_subdomains(const sf_context* c) { return c ? c->nsub : SF_ERR_INVALID; }

int sf_factor_fallbacks(const sf_context* c) { return c ? c->fp64_fallbacks : SF_ERR_INVALID; }

int sf_profile(sf_context* c, int32_t enable, double* ms, int64_t* launches) {
    if (!c) return SF_ERR_INVALID;
    SF_TRY(sfdd::prof_harvest(c));
    if (ms)
        for (int i = 0; i < 4; ++i) ms[i] = c->prof_ms[i];
    if (launches)
        for (int i = 0; i < 4; ++i) launches[i] = c->prof_n[i];
    if (enable >= 0) {
        c->profiling = enable ? 1 : 0;
        c->ev_used = 0;
        for (int i = 0; i < 4; ++i) {
            c->prof_ms[i] = 0.0;
            c->prof_n[i] = 0;
        }
    }
    return SF_OK;
}

int sf_memory_bytes(const sf_config* cfg, int64_t* bytes) {
    if (!cfg || !bytes) return SF_ERR_INVALID;
    SF_TRY(check_config(*cfg));
    std::vector<SubDesc> subs = plan_subdomains(*cfg);
    int maxmp = 0;
    for (const auto& d : subs) maxmp = std::max(maxmp, d.mp);
    if (maxmp > MAX_LINE) return SF_ERR_INVALID;
    int64_t fd = 0, wd = 0;
    storage_offsets(subs, cfg->factor_precision, &fd, &wd);
    *bytes = 8 * (fd + wd) + field_bytes(*cfg, (int64_t)subs.size());
    return SF_OK;
}

int sf_plan(const sf_config* cfg, int32_t* geom) {
    if (!cfg) return SF_ERR_INVALID;
    SF_TRY(check_config(*cfg));
    const std::vector<SubDesc> subs = plan_subdomains(*cfg);
    if (geom) {
        for (size_t i = 0; i < subs.size(); ++i) {
            const SubDesc& d = subs[i];
            int32_t* g = geom + 10 * i;
            g[0] = d.pair;
            g[1] = d.bx0;
            g[2] = d.bx0 + d.bw;
            g[3] = d.by0;
            g[4] = d.by0 + d.bh;
            g[5] = d.ox0;
            g[6] = d.ox1;
            g[7] = d.oy0;
            g[8] = d.oy1;
            g[9] = d.cols;
        }
    }
    return (int)subs.size();
}

int sf_subdomain_geometry(const sf_context* c, int32_t sub, int32_t* g) {
    if (!c || !g || sub < 0 || sub >= c->nsub) return SF_ERR_INVALID;
    const SubDesc& d = c->subs[sub];
    g[0] = d.pair;
    g[1] = d.bx0;
    g[2] = d.bx0 + d.bw;
    g[3] = d.by0;
    g[4] = d.by0 + d.bh;
    g[5] = d.ox0;
    g[6] = d.ox1;
    g[7] = d.oy0;
    g[8] = d.oy1;
    g[9] = d.cols;
    g[10] = d.P;
    g[11] = c->groups;
    g[12] = d.kmid;
    return SF_OK;
}

int sf_subdomain_solve(sf_context* c, int32_t sub, const double* b, double* x) {
    if (!c || !b || !x || sub < 0 || sub >= c->nsub || b == x) return SF_ERR_INVALID;
    SF_SETTLE(c);
    if (c->state != ST_FACTORED) return SF_ERR_STATE;
    SweepLock lock(c);
    hipLaunchKernelGGL(k_zero_status_api, dim3(1), dim3(1), 0, c->stream, c->status_d);
    SF_HIP(hipGetLastError());
    SF_TRY(sfdd::launch_sweep(c, nullptr, nullptr, sub, b, x));
    const int code = pull_status(c);
    return code;
}

}  // extern "C"

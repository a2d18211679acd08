// Internal types of the sfdd library (host and device).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "sfdd.h"

namespace sfdd {

constexpr int TS = 32;          // factor tile edge (doubles)
constexpr int TSZ = TS * TS;    // doubles per tile
constexpr int FACTOR_THREADS = 256;
constexpr int FACTOR_WS_SLOTS = 64;  // factor workspaces: subdomains per factor launch at most
constexpr int F2_MAX_NT = 24;        // cooperative factor: line matrices up to 768 x 768
constexpr int CLG_COEFS = 30;        // smoothed data-term coefficients per element (element.h)

// One subdomain: a box of the pixel grid cut into lines along its shorter side.
//   lines are columns (cols = 1): line t = x - bx0, position s = y - by0
//   lines are rows    (cols = 0): line t = y - by0, position s = x - bx0
// Local unknown 3*(t*ms + s) + c.  Line matrices are m x m (m = 3*ms),
// padded to mp = NT*TS for the tiled factor storage.
struct SubDesc {
    int32_t pair;
    int32_t bx0, by0, bw, bh;          // box origin and size (nodes)
    int32_t ox0, ox1, oy0, oy1;        // owned nodes, half-open global ranges
    int32_t cols;                      // 1: lines are columns
    int32_t ms, nt;                    // nodes per line, number of lines
    int32_t m, mp, NT, ntiles;         // line size, padded, tiles per side, tiles per line
    int32_t P;                         // workgroups per chain in a sweep
    int32_t kmid;                      // middle line of the twisted factorisation (nt - 1: one chain)
    int64_t foff;   // inverse Schur tiles: nt * ntiles * TSZ doubles
    int64_t boff;   // line couplings B_t: nt * m * 6 doubles (t = 0 unused)
    int64_t woff;   // sweep scratch: nt * mp doubles (forward results w_t)
    int64_t soff;   // factor workspace: max(3 mp^2, 2 (mp^2 + 2 NT TS^2)) doubles
    int64_t poff;   // sweep published rows: [2 chains][3 slots][mp] pairs of tagged 64-bit words
    int64_t aoff;   // line node blocks A[(t,s),(t,s)], A[(t,s),(t,s+1)]: nt * ms * 18 doubles
};

// Global node coordinates of local node (t, s).
__host__ __device__ inline void local_to_global(const SubDesc& d, int t, int s, int& x, int& y) {
    if (d.cols) { x = d.bx0 + t; y = d.by0 + s; }
    else        { x = d.bx0 + s; y = d.by0 + t; }
}

// Device-side status word (first error wins).
struct DevStatus {
    int32_t code;
    int32_t sub;
    int64_t row;
};

}  // namespace sfdd

struct sf_context {
    sf_config cfg;
    hipStream_t stream;
    int device;
    int W, H, B;
    int nsub;                       // over all pairs
    int state;                      // 0 created, 1 assembled, 2 factored
    int pending;                    // deferred status: PENDING_ASSEMBLE | PENDING_FACTOR
    long long wait_limit;           // unsuccessful polls of a device-side wait before it gives up
    std::vector<sfdd::SubDesc> subs;
    sfdd::SubDesc* d_subs;
    int maxP;                       // sweep workgroups per chain
    int sweep_capacity;             // co-resident sweep workgroups on the device
    int sweep_lanes;                // subdomains side by side in a sweep grid (8: each on one XCD)
    int sweep_chunk;                // subdomains per sweep launch
    int sweep_main;                 // of a launch's subdomains, at most this many side by side
                                    // (a multiple of sweep_lanes); the rest with contiguous ranks
    int groups;                     // chains per subdomain: 2 = twisted factorisation, 1 = top to bottom
    int sweep_rows;                 // largest number of block rows a sweep workgroup owns
    int factor_pf;                  // workgroups per subdomain in the cooperative factor (0: one-WG factor)
    int factor_chunk;               // subdomains per cooperative factor launch
    int factor_lanes;               // subdomains side by side in a factor grid (8: each on one XCD)
    int factor_main;                // of a launch's subdomains, at most this many side by side
                                    // (a multiple of factor_lanes); the rest with contiguous ranks
    uint32_t sweep_epoch;           // tag base for the sweep's published rows
    uint32_t factor_epoch;          // tag base for the factor's pivot blocks and inverses
    double* blur_w;                 // presmoothing weights, 2 blur_r + 1 (sigma > 0)
    int blur_r;
    double* clg_w;                  // K_rho weights, 2 clg_r + 1 (rho > 0)
    int clg_r;
    double* coef;                   // [B][30][ne] smoothed data-term coefficients (rho > 0), else null
    double* clg_tmp;                // [B][30][ne] first-pass sums (rho > 0)
    // per-pair field data
    double *f0, *ft, *alpha;        // [B][H][W], [B][H][W], [B][H-1][W-1][2]
    double *F, *r;                  // [B][3][H][W]
    double *eta;                    // [B][H-1][W-1][2] indicator scratch
    double *Fn2;                    // [B] ||F||^2
    double *Gn2;                    // [B] ||G||^2 of an adjoint right-hand side
    double *partials;               // reduction scratch
    int npart;                      // partial blocks per pair for node reductions
    double *relres_d;               // [B]
    int32_t *sweeps_d;              // [B]
    int32_t *done_d;                // [B]
    uint32_t *counters;             // [2 nsub] factor synchronisation, one per chain
    uint64_t *etamax_bits;          // [B]
    int32_t *flags_d;               // [4] input validation flags
    int32_t *fail_d;                // [nsub] subdomains whose factor met a rejected pivot
    int32_t *sublist_d;             // [1] the subdomain of a single-subdomain factor launch
    // subdomain storage
    double *factors;                // all subdomains' tiles and couplings
    double *work;                   // factor workspaces + sweep scratch
    int64_t factor_doubles, work_doubles;
    sfdd::DevStatus *status_d;
    sfdd::DevStatus status_h;       // last error detail
    // host staging (pinned)
    void *host_stage;
    // convergence checks of the Schwarz loop: two pinned slots of [status,
    // done flags [B]], each written behind its event, so that the host reads
    // one check while the iterations after it are already queued
    void *host_poll;
    hipEvent_t poll_ev[2];
    void *host_fail;                // [nsub] failure flags of the FP32 factorisation
    int fp64_fallbacks;             // subdomains of the last factorisation refactored in FP64
    // device address of the allocation-free entry point's static scratch array
    double *scratch;
    // graph-replayed Schwarz loop (sf_schwarz_solve_graph): a private stream,
    // and the iteration index and sweep tag base kept on the device so that a
    // replayed graph reads fresh values
    hipStream_t gstream;            // created on first use: default priority, non-blocking
    hipEvent_t gev[2];
    int32_t *gk_d;                  // iteration index read by the convergence test
    uint32_t *gepoch_d;             // tag base read by the sweep
    int graph_capture;              // 1 while the chunk graph is being captured
    // optional per-kernel timing (sf_profile): event pairs around launches
    int profiling;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kind;       // kernel class of each pending pair
    int ev_used;
    double prof_ms[4];
    int64_t prof_n[4];
};

// kernel launchers (fem.hip, factor.hip, solve.hip)
namespace sfdd {
int launch_validate(sf_context* c, const double* I0, const double* I1, const double* alpha);
int launch_assemble(sf_context* c, const double* I0, const double* I1, const double* alpha);
int launch_presmooth(sf_context* c, const double* I, double* out, double* tmp);
int launch_clg(sf_context* c);
int launch_residual(sf_context* c, const double* U, double* r, int fuse_converge, double rtol, int sweep,
                    int max_sweeps, const double* rhs = nullptr, const double* rhs_n2 = nullptr);
int launch_norm2(sf_context* c, const double* G, double* out);
int launch_zero_where_rhs_zero(sf_context* c, double* U, const double* rhs_n2);
int launch_adjoint_gradients(sf_context* c, const double* U, const double* P, double* dI0, double* dI1,
                             double* dal);
int launch_indicator(sf_context* c, const double* U, double* eta, int reset_max);
int scratch_resolve(int device, double** out);
int64_t scratch_residual_doubles(const sf_context* c);
int launch_residual_scratch(sf_context* c, const double* U, double* r, double* scr);
int launch_alpha_update(sf_context* c, const double* eta, double* alpha_out, double kappa,
                        double eta_thr, double alpha_th);
int launch_factor(sf_context* c);
int launch_factor2(sf_context* c, int sub0, int nsub_chunk, int Pf, int fp32_arith, const int32_t* sublist,
                   int lanes, int main_cap, double ptol);
int launch_line_coeffs(sf_context* c);
const void* factor2_kernel(int fp32);
int launch_sweep(sf_context* c, double* U, const double* r, int single_sub, const double* b_local,
                 double* x_local);
uint32_t sweep_epoch_step(const sf_context* c);   // tag base advance of one sweep launch
enum { SWEEP_GENERAL = 0, SWEEP_FAST2 = 1, SWEEP_FAST1 = 2 };
const void* sweep_kernel(int form, int fp32);
int sweep_threads(int form);
int sweep_form(const sf_context* c);
// timing helpers (api.hip): bracket a launch of kernel class `kind`
int prof_begin(sf_context* c, int kind);
int prof_end(sf_context* c);
int prof_harvest(sf_context* c);
enum { PROF_SWEEP = 0, PROF_FACTOR = 1, PROF_RESIDUAL = 2, PROF_OTHER = 3 };
}  // namespace sfdd

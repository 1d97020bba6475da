// tsspin.cpp -- C ABI of libtsspin: argument checks, the Hamiltonian tables, plan cache
// and kernel dispatch.  See include/tsspin.h for the contract of every entry point.
#include "../../include/tsspin.h"

#include <hip/hip_runtime_api.h>

#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cctype>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

ts_status fail(ts_status st, const std::string &msg)
{
    g_err = msg;
    return st;
}

#define TS_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(TS_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxSpinsC128 = 34;
constexpr int kAdjMinSpins = 8;
constexpr int kMaxBatchPrograms = 8;   // captured batch programs kept per context   // the adjoint's sweeps need tiles of at least 2^8 amplitudes
constexpr int kMaxSpinsC64 = 35;

// 2^12-amplitude tiles: two (complex128) or four (complex64) workgroups per CU by LDS, and
// at N = 27 still three bit groups (two sweeps per layer) with runs of >= 256 bytes.
int default_tile_bits(int dtype) { (void)dtype; return 12; }
int min_run_bits(int dtype) { return dtype == TS_C128 ? 3 : 4; }  // 128-byte runs
// Light-cone sweeps: low memory bits kept in every tile (runs of 16 amplitudes).
constexpr int kConeLowBits = 4;
bool valid_config(int dtype, int n, int T, int RB, int variant);

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

// Energy tables of one (tile layout, axis): per-workgroup outside energy and effective
// fields, and the tile-internal couplings.
struct EnergyTable {
    DevBuf wg, jt;
    std::vector<double> wg_host;   // host copy of wg, for the phase-factor tables
};

struct PlanEntry {
    ts::Plan plan;
    DevBuf resident_ops;   // ResidentOp[] when plan.resident
    // one vector's resident ops with precomputed phase factors (N <= 13): the factors of the
    // distinct phase steps, those steps' ops, and the op list that points at the factors
    DevBuf resident_fac, resident_uniq, resident_fac_ops;
    std::vector<tsk::DiagArgs> diag_args;  // one per chain diagonal
    bool prepared = false;                 // launch arguments below are built
    int reg_bits = 0;
    std::vector<tsk::SweepArgs> lds_args;
    std::vector<tsk::RegSweepArgs> reg_args;
    // light-cone form of the same run (used instead of `plan` when `cone` is set)
    bool cone = false;
    double cone_cost = 0.0;                // the cost model's time of the light-cone form (us)
    ts::ConePlan cone_plan;
    DevBuf cone_dev;                       // tsk::ConeArgs[] of every sweep
    std::vector<tsk::ConeArgs> cone_host;  // host copy (batched launches gather them)
    bool cone_prepared = false;
    std::vector<std::vector<int>> cone_phase_win;  // register window of each phase step, per sweep
    // adjoint plans: the light-cone form (looked for once) and its gradient terms
    bool cone_tried = false;
    bool cone_grad_prepared = false, cone_grad_ok = false;
    DevBuf cone_grad_dev;                  // tsk::ConeGradArgs[] of every sweep
    std::vector<int> cone_grad_slots;      // accumulators of each sweep
    // energy-table variant: table pointers and phase-layout offsets filled in reg_args
    bool etab_prepared = false, etab_ok = false;
};

// Phase factors of one light-cone phase step (restricted terms): workgroup rows and the
// per-thread / window table.
struct ConeTab {
    DevBuf wgf, dtab;
    int8_t row_bit[tsk::kConeRowBits] = {};
    int n_row_bits = 0;
    uint32_t xmask = 0;   // tile bits with a row-dependent field
    uint32_t cmask = 0;   // window bits with a thread- or workgroup-dependent walk factor
};

}  // namespace

struct ts_ctx {
    int n = 0;
    std::vector<int> bi, bj;                    // merged bonds, bi < bj
    std::vector<std::array<double, 3>> J;       // merged couplings
    std::vector<std::array<double, 3>> h;       // fields [n]
    std::vector<int> input_bond;                // input bond k -> merged bond index
    bool zero_axis[3] = {false, false, false};
    int device = -1;
    int tile_bits[2] = {0, 0};                  // per dtype, 0 = default
    // per dtype: 0 register-window, 1 LDS-staged, 2 pipelined, 3 register-window with the
    // half-LDS complex128 kernel on the top bit group, 4 light-cone sweeps where the cost
    // model prefers them, else the ping-pong sweeps of 3 (complex128) or 0 (complex64)
    int sweep_variant[2] = {4, 4};
    int reg_bits[2] = {4, 4};                   // per dtype: amplitudes per thread = 2^RB
    bool balance = true;                        // plans move shared low-bit rotations off phase sweeps
    // light-cone sweeps: -1 as the sweep variant says, 0 never, 1 where the cost model
    // prefers them, 2 wherever they fit the kernel
    int cone_mode = -1;
    int cone_adv = 0;                           // layers one spin may take per light-cone sweep (0: any)
    double watchdog = -1.0;                     // ts_evolve norm-drift bound (< 0: off)
    DevBuf watch_buf;                           // norms before and after, [2][n_psi]
    std::map<std::string, std::unique_ptr<ConeTab>> cone_tabs;
    bool tune_checked[2] = {false, false};      // tuning cache consulted for this dtype
    bool user_config[2] = {false, false};       // tile width set explicitly: keep it
    std::map<std::tuple<int, uint64_t, int>, std::unique_ptr<EnergyTable>> tables;
    std::map<std::tuple<int, int, int, uint64_t, int64_t>, std::unique_ptr<PlanEntry>> plans;
    std::map<std::tuple<int, uint64_t, int, uint64_t, int, int>, std::unique_ptr<DevBuf>> diag_tabs;
    std::map<std::tuple<int, uint64_t, int, uint64_t>, std::unique_ptr<DevBuf>> wgf_tabs;
    DevBuf partials;       // reduction scratch
    DevBuf cone_partials;  // observables folded into light-cone sweeps: [workgroups][2 * kMaxObs]
    int64_t cone_partial_rows = 0;   // workgroups of the last sweep that wrote them
    bool no_fuse = false;  // $TSSPIN_NO_FUSE: records always by separate reductions
    bool res_fac = true;   // $TSSPIN_RESIDENT_FACTORS=0: resident ops form their phases in place
    bool adj_split = false;  // $TSSPIN_ADJ_SPLIT: the adjoint's split-phase plan and separate gradient passes
    bool adj_cone = true;    // $TSSPIN_ADJ_CONE=0: the adjoint's reverse pass keeps the ping-pong form
    DevBuf expect_out;     // ts_expect staging
    DevBuf grad_acc;       // ts_adjoint gradients [3][n + bonds]
    DevBuf grad_slots;     // ts_adjoint per-workgroup accumulators [workgroups][3][n + bonds]
    DevBuf grad_explicit;  // ts_adjoint, energy loss: <dH/dtheta> at the final state [3][n + bonds]
    DevBuf grad_params;    // ts_adjoint: spins and columns of every parameter, grouped for grad_walsh_kernel
    // ts_adjoint below kAdjMinSpins: the same problem on that many spins, and its state,
    // input and workspace
    std::unique_ptr<ts_ctx> adj_pad;
    DevBuf adj_pad_buf;
    DevBuf unit_phase;     // one (1, 0) factor row for sweeps whose phase step has no energy
    DevBuf etab[2][3];     // energy tables D_axis(b) per dtype (double / float) and axis
    DevBuf ham_h, ham_b;   // fields [n][3] and merged bonds (tsk::HamBond) for the energy
    // batch context: one sub-context per chain (empty for a single system)
    std::vector<std::unique_ptr<ts_ctx>> chains;
    std::map<std::string, std::unique_ptr<struct BatchProgram>> programs;
    std::vector<std::string> program_order;     // keys of `programs`, least recently used first
    int64_t graph_replays = 0, eager_runs = 0, capture_failures = 0;
    ~ts_ctx();
};

namespace {

ts_status ensure_device(ts_ctx *c)
{
    int dev = 0;
    TS_HIP(hipGetDevice(&dev));
    if (c->device >= 0 && c->device != dev)
        return fail(TS_EINVAL, "context was first used on another device");
    c->device = dev;
    return TS_OK;
}

ts_status alloc(DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes && b.p) return TS_OK;
    if (b.p) {
        TS_HIP(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return fail(e == hipErrorOutOfMemory ? TS_ENOMEM : TS_EDEVICE,
                    std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    b.bytes = bytes;
    return TS_OK;
}

inline double spin(uint64_t b, int j) { return ((b >> j) & 1) ? 0.5 : -0.5; }

// Tables for the tile layout `tile` (T bits) of an n-spin register, axis a.
ts_status get_table(ts_ctx *c, int T, uint64_t tile, int axis, EnergyTable **out)
{
    auto key = std::make_tuple(T, tile, axis);
    auto it = c->tables.find(key);
    if (it != c->tables.end()) {
        *out = it->second.get();
        return TS_OK;
    }
    const int n = c->n;
    const uint64_t all = (1ull << n) - 1;
    const uint64_t outside = all & ~tile;
    int pos[64];
    int kof[64];
    int Tk = 0;
    for (int b = 0; b < n; ++b) {
        kof[b] = -1;
        if ((tile >> b) & 1) {
            kof[b] = Tk;
            pos[Tk++] = b;
        }
    }
    const int nout = n - Tk;
    const uint64_t nwg = 1ull << nout;
    std::vector<double> wg((size_t)nwg * (T + 1), 0.0), jt((size_t)T * T, 0.0);
    for (size_t k = 0; k < c->bi.size(); ++k) {
        const int p = c->bi[k], q = c->bj[k];
        if (kof[p] >= 0 && kof[q] >= 0) {
            int k1 = kof[p], k2 = kof[q];
            if (k1 > k2) std::swap(k1, k2);
            jt[(size_t)k1 * T + k2] += c->J[k][axis];
        }
    }
    for (uint64_t w = 0; w < nwg; ++w) {
        const uint64_t base = ts::deposit(w, outside);
        double *row = &wg[(size_t)w * (T + 1)];
        double C = 0.0;
        for (int j = 0; j < n; ++j) {
            const double hj = c->h[j][axis];
            if (kof[j] >= 0) row[1 + kof[j]] += hj;
            else C += hj * spin(base, j);
        }
        for (size_t k = 0; k < c->bi.size(); ++k) {
            const int p = c->bi[k], q = c->bj[k];
            const double Jk = c->J[k][axis];
            const bool pi = kof[p] >= 0, qi = kof[q] >= 0;
            if (!pi && !qi) C += Jk * spin(base, p) * spin(base, q);
            else if (pi && !qi) row[1 + kof[p]] += Jk * spin(base, q);
            else if (!pi && qi) row[1 + kof[q]] += Jk * spin(base, p);
        }
        row[0] = C;
    }
    auto t = std::make_unique<EnergyTable>();
    ts_status st = alloc(t->wg, wg.size() * sizeof(double));
    if (st != TS_OK) return st;
    st = alloc(t->jt, jt.size() * sizeof(double));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(t->wg.p, wg.data(), wg.size() * sizeof(double), hipMemcpyHostToDevice));
    TS_HIP(hipMemcpy(t->jt.p, jt.data(), jt.size() * sizeof(double), hipMemcpyHostToDevice));
    t->wg_host.swap(wg);
    *out = t.get();
    c->tables.emplace(key, std::move(t));
    return TS_OK;
}

// Workgroup phase factors of one (tile layout, axis, tau): per tile, exp(-i tau C) and then
// exp(-i tau geff_k / 2) for every tile bit k, as (re, im) pairs [tiles][T+1].  C and geff
// are the outside energy and effective fields of the energy table.
ts_status get_wgf_table(ts_ctx *c, int T, uint64_t tile, int axis, double tau, const double **out)
{
    uint64_t tb;
    std::memcpy(&tb, &tau, sizeof tb);
    auto key = std::make_tuple(T, tile, axis, tb);
    auto it = c->wgf_tabs.find(key);
    if (it != c->wgf_tabs.end()) {
        *out = static_cast<const double *>(it->second->p);
        return TS_OK;
    }
    EnergyTable *et;
    ts_status st = get_table(c, T, tile, axis, &et);
    if (st != TS_OK) return st;
    const std::vector<double> &wg = et->wg_host;
    std::vector<double> f(2 * wg.size());
    for (size_t i = 0; i < wg.size(); ++i) {
        const double e = (i % (size_t)(T + 1)) ? 0.5 * wg[i] : wg[i];
        f[2 * i] = std::cos(tau * e);
        f[2 * i + 1] = -std::sin(tau * e);
    }
    auto buf = std::make_unique<DevBuf>();
    st = alloc(*buf, f.size() * sizeof(double));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(buf->p, f.data(), f.size() * sizeof(double), hipMemcpyHostToDevice));
    *out = static_cast<const double *>(buf->p);
    c->wgf_tabs.emplace(key, std::move(buf));
    return TS_OK;
}

tsk::DiagArgs diag_args(const ts::DiagStep &d)
{
    tsk::DiagArgs a;
    a.axis = d.axis;
    a.qturn = d.qturn;
    a.tau = d.tau;
    double mag = std::ldexp(1.0, -d.mag_exp);
    if (d.mag_sqrt) mag *= 0.70710678118654752440;
    // exp(i pi k / 4), exact on the axes
    static const double r = 0.70710678118654752440;
    const double cs[8] = {1, r, 0, -r, -1, -r, 0, r};
    const double sn[8] = {0, r, 1, r, 0, -r, -1, -r};
    a.kre = mag * cs[d.eighths & 7];
    a.kim = mag * sn[d.eighths & 7];
    return a;
}

// Light-cone plan of the same chain, kept when the cost model prefers it over the ping-pong
// plan (mode 1) or whenever it fits the kernel (mode 2).  Model (fitted to kernel traces of
// the xyz chain at N = 27, in microseconds for 2^27 amplitudes; within 4% at N = 27 and 30):
// a light-cone sweep costs 526 + 30.3 per transpose + 40.1 per phase step + 11.3 per
// spin-layer (complex128) or 201 + 8.3 + 41.5 + 11.9 (complex64): it is bound by latency,
// vector instructions and LDS, not by HBM.  A ping-pong sweep moves the state once: see
// pingpong_sweep_us.  Both scale with 2^(N-27); every launch adds about 8 us, which decides
// at small N.
double pingpong_sweep_us(int dtype, int T)
{
    // measured per sweep at N = 27 (complex64 T = 13, 14 and complex128 T = 13: N = 27-30)
    if (dtype == TS_C128) return T >= 13 ? 1000.0 : 790.0;
    return T >= 14 ? 550.0 : T == 13 ? 480.0 : 415.0;
}
bool cone_stages(const ts::ConeSweep &sw, int T, int RB, int s, tsk::ConeArgs &a,
                 std::vector<int> &phase_win, int *transposes);

bool cone_candidate(ts_ctx *c, PlanEntry *pe, int T, int dtype, int mode)
{
    std::vector<std::pair<int, int>> bonds;
    for (size_t k = 0; k < c->bi.size(); ++k) bonds.push_back({c->bi[k], c->bj[k]});
    ts::ConePlan cp;
    const size_t limit = 4 * pe->plan.sweeps.size() + 16;
    if (!ts::make_cone_plan(pe->plan.chain, c->n, T, kConeLowBits, bonds, c->cone_adv, limit, cp,
                            tsk::kConePhases))
        return false;
    double cost = 0.0;
    for (const ts::ConeSweep &sw : cp.sweeps) {
        tsk::ConeArgs a;
        std::vector<int> pw;
        int tr = 0;
        if (sw.phases.size() > (size_t)tsk::kConePhases || !cone_stages(sw, T, 4, kConeLowBits, a, pw, &tr))
            return false;  // does not fit the kernel's limits: keep the ping-pong plan
        // a phase step selects its workgroup row by the bits of the outside spins its
        // bonds reach; the kernel holds kConeRowBits of them
        std::vector<char> in_tile(c->n, 0);
        for (int q : sw.tile_q) in_tile[q] = 1;
        for (const ts::ConePhase &ph : sw.phases) {
            uint64_t outside = 0;
            for (int b : ph.bonds) {
                const int p = c->bi[b], q = c->bj[b];
                if (in_tile[p] != in_tile[q]) outside |= 1ull << (in_tile[p] ? q : p);
            }
            if (__builtin_popcountll(outside) > tsk::kConeRowBits) return false;
        }
        int sl = 0;
        for (const ts::ConeOp &op : sw.ops)
            if (op.kind == 0) sl += __builtin_popcountll(op.spins);
        const double ph = (double)sw.phases.size();
        cost += dtype == TS_C128 ? 526.0 + 30.3 * tr + 40.1 * ph + 11.3 * sl
                                 : 201.0 + 8.3 * tr + 41.5 * ph + 11.9 * sl;
    }
    const double pp = (double)pe->plan.sweeps.size() * pingpong_sweep_us(dtype, T);
    const double scale = std::ldexp(1.0, c->n - 27), launch = 8.0;
    cost = cost * scale + launch * (double)cp.sweeps.size();
    const double ppc = pp * scale + launch * (double)pe->plan.sweeps.size();
    if (mode == 1 && cost >= 0.95 * ppc) return false;
    pe->cone_plan = std::move(cp);
    pe->cone_cost = cost;
    return true;
}

// adjoint = true: keep the partial evolutions of vanishing axes (their parameters still
// have gradients) and end a sweep at every phase step (split_phases).
// adjoint: the inverse chain with every axis kept; split additionally ends a sweep at each
// phase step (for the adjoint's separate gradient pass).
ts_status build_plan(ts_ctx *c, int dtype, int T, int order, double dt, int64_t nsteps,
                     PlanEntry **out, bool adjoint = false, bool split = true)
{
    uint64_t dtb;
    std::memcpy(&dtb, &dt, sizeof dtb);
    auto key = std::make_tuple(dtype + (adjoint ? (split ? 2 : 4) : 0), T, order, dtb, nsteps);
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second.get();
        return TS_OK;
    }
    auto pe = std::make_unique<PlanEntry>();
    try {
        const bool none[3] = {false, false, false};
        // the adjoint plan is the exact inverse of the forward run with step dt
        auto chain = ts::build_chain(order, dt, nsteps, adjoint ? none : c->zero_axis, adjoint);
        pe->plan = ts::make_plan(chain, c->n, T, min_run_bits(dtype), adjoint && split, c->balance);
    } catch (const std::exception &e) {
        return fail(TS_EINVAL, std::string("plan: ") + e.what());
    }
    for (const auto &d : pe->plan.chain.diags) pe->diag_args.push_back(diag_args(d));
    const int cm = c->cone_mode >= 0 ? c->cone_mode : (c->sweep_variant[dtype] == 4 ? 1 : 0);
    if (!adjoint && cm > 0 && !pe->plan.resident && c->reg_bits[dtype] == 4 && (T == 11 || T == 12))
        pe->cone = cone_candidate(c, pe.get(), T, dtype, cm);
    *out = pe.get();
    c->plans.emplace(key, std::move(pe));
    return TS_OK;
}

// Tile width of ts_evolve when the caller fixed none.  The default (12) keeps every tile
// wide enough for runs of >= 128 bytes and lets several workgroups share a CU; a wider
// tile is taken when it cuts the bit groups of the ping-pong sweeps (one sweep fewer per
// layer for each group saved: the 5 x 6 dipolar lattice in complex64 needs 4 groups at 12
// and 3 at 13, 61 instead of 41 sweeps per step), unless the light-cone form, which runs at
// the default width, is faster by the cost model than the wider ping-pong plan.
ts_status resolve_tile(ts_ctx *c, int dtype, int order, double dt, int64_t nsteps, int *T_out)
{
    const int T0 = c->tile_bits[dtype] > 0 ? c->tile_bits[dtype] : default_tile_bits(dtype);
    *T_out = T0;
    if (c->tile_bits[dtype] > 0 || c->n <= T0) return TS_OK;
    auto ngroups = [&](int T) {
        std::vector<uint64_t> g, t;
        ts::plan_groups(c->n, T, min_run_bits(dtype), g, t);
        return g.size();
    };
    int best = T0;
    size_t gbest = ngroups(T0);
    for (int T = T0 + 1; T <= (dtype == TS_C128 ? 13 : 14) && T < c->n; ++T) {
        const size_t g = ngroups(T);
        if (g < gbest) best = T, gbest = g;
    }
    if (best == T0) return TS_OK;
    PlanEntry *p0, *pw;
    ts_status st = build_plan(c, dtype, T0, order, dt, nsteps, &p0);
    if (st != TS_OK) return st;
    st = build_plan(c, dtype, best, order, dt, nsteps, &pw);
    if (st != TS_OK) return st;
    if (p0->cone && c->cone_mode == 2) return TS_OK;   // light-cone sweeps wherever they fit
    if (p0->cone) {
        const double ppw = (double)pw->plan.sweeps.size() *
                           (pingpong_sweep_us(dtype, best) * std::ldexp(1.0, c->n - 27) + 8.0);
        if (p0->cone_cost < 0.95 * ppw) return TS_OK;
    }
    *T_out = best;
    return TS_OK;
}

// Upload the resident op list (needs the device).
ts_status resident_ops(PlanEntry *pe)
{
    if (pe->resident_ops.p) return TS_OK;
    std::vector<tsk::ResidentOp> ops;
    for (const auto &s : pe->plan.sweeps) {
        tsk::ResidentOp op{};
        op.d = s.diag >= 0 ? pe->diag_args[s.diag] : tsk::DiagArgs{-1, 0, 0.0, 1.0, 0.0};
        op.post = s.post_mask != 0;
        op.rec = -1;
        ops.push_back(op);
    }
    ts_status st = alloc(pe->resident_ops, ops.size() * sizeof(tsk::ResidentOp));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(pe->resident_ops.p, ops.data(), ops.size() * sizeof(tsk::ResidentOp),
                     hipMemcpyHostToDevice));
    return TS_OK;
}

bool fill_runs(uint64_t mask, tsk::Run *runs, int32_t *nruns)
{
    auto rs = ts::deposit_runs(mask);
    if (rs.size() > 4) return false;  // the kernel argument holds four runs
    *nruns = (int32_t)rs.size();
    for (size_t i = 0; i < rs.size(); ++i)
        runs[i] = tsk::Run{(int8_t)rs[i].src, (int8_t)rs[i].len, (int8_t)rs[i].dst, 0};
    return true;
}

// Map a global-bit mask onto tile-index bits.
uint32_t to_tile_bits(uint64_t mask, uint64_t tile)
{
    uint32_t r = 0;
    int k = 0;
    for (int b = 0; b < 64; ++b) {
        if (!((tile >> b) & 1)) continue;
        if ((mask >> b) & 1) r |= 1u << k;
        ++k;
    }
    return r;
}

// Phase factors of one phase step of the register-window sweep that depend only on the
// thread's tile bits (not on the workgroup), for the tile layout `tile`, axis, tau, the
// quarter-turn count c and the register window [w, w+RB):
//   per thread pattern t0 (window bits zero):
//     [0]    i^(c*popcount(t0)) * exp(-i tau sum_{k1<k2 outside window} J s_k1 s_k2)
//     [1+v]  exp(-i tau h_v / 2),  h_v = sum_{k outside window} J_{k,w+v} s_k
//   then q[r] = i^(c*popcount(r)) * exp(-i tau sum_{v1<v2} J_{w+v1,w+v2} s_v1 s_v2).
ts_status get_diag_table(ts_ctx *c, int T, int RB, uint64_t tile, int axis, double tau, int qturn,
                         int w, const double **out)
{
    uint64_t tb;
    std::memcpy(&tb, &tau, sizeof tb);
    auto key = std::make_tuple(T * 16 + RB, tile, axis, tb, qturn, w);
    auto it = c->diag_tabs.find(key);
    if (it != c->diag_tabs.end()) {
        *out = static_cast<const double *>(it->second->p);
        return TS_OK;
    }
    int kof[64];
    int Tk = 0;
    for (int b = 0; b < c->n; ++b) kof[b] = ((tile >> b) & 1) ? Tk++ : -1;
    std::vector<double> Jt((size_t)T * T, 0.0);
    if (axis < 3) {
        for (size_t k = 0; k < c->bi.size(); ++k) {
            const int p = kof[c->bi[k]], q = kof[c->bj[k]];
            if (p >= 0 && q >= 0) Jt[(size_t)std::min(p, q) * T + std::max(p, q)] += c->J[k][axis];
        }
    }
    auto J = [&](int a, int b) { return a < b ? Jt[(size_t)a * T + b] : Jt[(size_t)b * T + a]; };
    auto s = [](uint32_t t, int k) { return ((t >> k) & 1) ? 0.5 : -0.5; };
    auto qt = [](int m) {
        static const ts::cplx q[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
        return q[m & 3];
    };
    auto ex = [&](double e) { return ts::cplx(std::cos(tau * e), -std::sin(tau * e)); };
    auto in_win = [&](int k) { return k >= w && k < w + RB; };
    const int nthr = 1 << (T - RB);
    std::vector<ts::cplx> tab((size_t)nthr * (1 + RB) + (1u << RB));
    for (int tid = 0; tid < nthr; ++tid) {
        const uint32_t t0 = (tid & ((1u << w) - 1u)) | ((uint32_t)(tid >> w) << (w + RB));
        double e = 0.0;
        for (int k1 = 0; k1 < T; ++k1)
            for (int k2 = k1 + 1; k2 < T; ++k2)
                if (!in_win(k1) && !in_win(k2)) e += J(k1, k2) * s(t0, k1) * s(t0, k2);
        tab[(size_t)tid * (1 + RB)] = qt(qturn * __builtin_popcount(t0)) * ex(e);
        for (int v = 0; v < RB; ++v) {
            double h = 0.0;
            for (int k = 0; k < T; ++k)
                if (!in_win(k)) h += J(k, w + v) * s(t0, k);
            tab[(size_t)tid * (1 + RB) + 1 + v] = ex(0.5 * h);
        }
    }
    for (uint32_t r = 0; r < (1u << RB); ++r) {
        double e = 0.0;
        for (int v1 = 0; v1 < RB; ++v1)
            for (int v2 = v1 + 1; v2 < RB; ++v2) e += J(w + v1, w + v2) * s(r, v1) * s(r, v2);
        tab[(size_t)nthr * (1 + RB) + r] = qt(qturn * __builtin_popcount(r)) * ex(e);
    }
    auto buf = std::make_unique<DevBuf>();
    ts_status st = alloc(*buf, tab.size() * sizeof(ts::cplx));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(buf->p, tab.data(), tab.size() * sizeof(ts::cplx), hipMemcpyHostToDevice));
    *out = static_cast<const double *>(buf->p);
    c->diag_tabs.emplace(key, std::move(buf));
    return TS_OK;
}

// Stage list of the register-window sweep for one pass.  A window is RB consecutive tile
// bits [w, w + RB): each thread holds the 2^RB amplitudes along it, and moving to another
// window costs one LDS transpose.  The pre bits are rotated first, in any window order
// (rotations of distinct bits commute), then the phase step runs in the window where they
// end, then the post bits.  Load and store use windows at or above s_min, so that lanes
// carry the low (contiguous) index bits.  A memoised search over (window, bits left) finds
// an order with the fewest transposes.  In each window visited every bit of the current
// part that it holds is rotated, so every bit is rotated exactly once.
bool search_stages(int T, int RB, uint32_t pre, uint32_t post, bool diag, int s_min,
                   tsk::RegSweepArgs &a);

// Long plans repeat a handful of (pre, post, phase) patterns: the search runs once per
// pattern and the result is reused (process-wide, guarded).
bool make_stages(int T, int RB, uint32_t pre, uint32_t post, bool diag, int s_min,
                 tsk::RegSweepArgs &a)
{
    struct Prog {
        bool ok;
        uint64_t code[2];
        int32_t n, load, store, diag;
    };
    static std::mutex mu;
    static std::map<std::tuple<int, int, uint32_t, uint32_t, bool, int>, Prog> cache;
    const auto key = std::make_tuple(T, RB, pre, post, diag, s_min);
    {
        std::lock_guard<std::mutex> lk(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            const Prog &p = it->second;
            a.st_code[0] = p.code[0];
            a.st_code[1] = p.code[1];
            a.n_stages = p.n;
            a.load_win = p.load;
            a.store_win = p.store;
            a.diag_win = p.diag;
            return p.ok;
        }
    }
    const bool ok = search_stages(T, RB, pre, post, diag, s_min, a);
    std::lock_guard<std::mutex> lk(mu);
    cache[key] = Prog{ok, {a.st_code[0], a.st_code[1]}, a.n_stages, a.load_win, a.store_win, a.diag_win};
    return ok;
}

bool search_stages(int T, int RB, uint32_t pre, uint32_t post, bool diag, int s_min,
                   tsk::RegSweepArgs &a)
{
    const int top = T - RB;
    if (top < 0 || top > 15 || RB > 4 || T > 16) return false;
    if ((pre | post) & ~((1u << T) - 1u)) return false;
    s_min = std::min(s_min, top);
    auto wmask = [&](int w) { return ((1u << RB) - 1u) << w; };
    // memo[part][(w, bits left after w)] = (transposes to the end, next window)
    std::map<uint64_t, std::pair<int, int>> memo[2];
    std::function<int(int, int, uint32_t)> cost = [&](int part, int w, uint32_t rem) -> int {
        rem &= ~wmask(w);
        const uint64_t key = ((uint64_t)w << 32) | rem;
        auto it = memo[part].find(key);
        if (it != memo[part].end()) return it->second.first;
        int best = INT_MAX, next = -1;
        if (rem == 0) {
            best = part == 0 ? cost(1, w, post) : (w >= s_min ? 0 : 1);
        } else {
            for (int v = top; v >= 0; --v) {
                if (v == w || !(rem & wmask(v))) continue;
                const int c = 1 + cost(part, v, rem);
                if (c < best) {
                    best = c;
                    next = v;
                }
            }
        }
        memo[part][key] = {best, next};
        return best;
    };
    int start = top, best = INT_MAX;
    for (int s = top; s >= s_min; --s) {
        const int c = cost(0, s, pre);
        if (c < best) {
            best = c;
            start = s;
        }
    }
    int ns = 0;
    a.st_code[0] = a.st_code[1] = 0;
    auto push = [&](int w, uint32_t m, int op) {
        if (ns >= tsk::kMaxStages) return false;
        a.st_code[ns / tsk::kStagesPerWord] |= (uint64_t)tsk::stage_code(w, op, m)
                                               << (9 * (ns % tsk::kStagesPerWord));
        ++ns;
        return true;
    };
    a.diag_win = -1;
    int w = start, part = 0;
    uint32_t rem = pre;
    for (;;) {
        const uint32_t b = rem & wmask(w);
        if (b) {
            if (!push(w, b >> w, 0)) return false;
            rem &= ~b;
        }
        if (rem) {
            w = memo[part].at(((uint64_t)w << 32) | rem).second;
            if (w < 0) return false;
            continue;
        }
        if (part == 1) break;
        if (diag) {
            if (!push(w, 0, 1)) return false;
            a.diag_win = w;
        }
        part = 1;
        rem = post;
    }
    a.n_stages = ns;
    a.load_win = start;
    a.store_win = w >= s_min ? w : top;
    return true;
}

// Bits by which the order of strided tiles is rotated (RegSweepArgs::rot), and the state
// size from which they are (the N = 30 lattice, 8 GiB: 4.8% faster rotated).
constexpr int kTileRot = 5;
constexpr size_t kTileRotBytes = (size_t)4 << 30;

// Launch arguments of every sweep of a tiled plan, built once per plan (tables included).
ts_status prepare_sweeps(ts_ctx *c, PlanEntry *pe, int dtype)
{
    if (pe->prepared && pe->reg_bits == c->reg_bits[dtype]) return TS_OK;
    const ts::Plan &P = pe->plan;
    const int n = c->n;
    const int T = P.tile_bits;
    const int RB = c->reg_bits[dtype];
    const uint64_t all = (1ull << n) - 1;
    pe->lds_args.clear();
    pe->reg_args.clear();
    pe->etab_prepared = false;
    for (const ts::Sweep &sw : P.sweeps) {
        tsk::SweepArgs a{};
        if (!fill_runs(sw.tile_mask, a.tile_runs, &a.n_tile_runs) ||
            !fill_runs(all & ~sw.tile_mask, a.out_runs, &a.n_out_runs))
            return fail(TS_EINVAL, "internal: tile layout has more than four bit runs");
        if (__builtin_popcountll(sw.tile_mask) != T || (sw.tile_mask & ~all))
            return fail(TS_EINVAL, "internal: tile mask does not match the tile width");
        a.pre_mask = to_tile_bits(sw.pre_mask, sw.tile_mask);
        a.post_mask = to_tile_bits(sw.post_mask, sw.tile_mask);
        a.d = sw.diag >= 0 ? pe->diag_args[sw.diag] : tsk::DiagArgs{-1, 0, 0.0, 1.0, 0.0};
        if (a.d.axis >= 0 && a.d.axis < 3) {
            EnergyTable *t;
            ts_status st = get_table(c, T, sw.tile_mask, a.d.axis, &t);
            if (st != TS_OK) return st;
            a.wg = static_cast<const double *>(t->wg.p);
            a.jt = static_cast<const double *>(t->jt.p);
        }
        pe->lds_args.push_back(a);
        tsk::RegSweepArgs r{};
        std::memcpy(r.tile_runs, a.tile_runs, sizeof r.tile_runs);
        std::memcpy(r.out_runs, a.out_runs, sizeof r.out_runs);
        r.n_tile_runs = a.n_tile_runs;
        r.n_out_runs = a.n_out_runs;
        r.d = a.d;
        r.jt = a.jt;
        if (a.d.axis >= 0 && a.d.axis < 3) {
            ts_status st = get_wgf_table(c, T, sw.tile_mask, a.d.axis, a.d.tau, &r.wgf);
            if (st != TS_OK) return st;
        } else {
            if (!c->unit_phase.p) {
                const double one[2] = {1.0, 0.0};
                ts_status st = alloc(c->unit_phase, sizeof one);
                if (st != TS_OK) return st;
                TS_HIP(hipMemcpy(c->unit_phase.p, one, sizeof one, hipMemcpyHostToDevice));
            }
            r.wgf = static_cast<const double *>(c->unit_phase.p);
        }
        if (!make_stages(T, RB, a.pre_mask, a.post_mask, a.d.axis >= 0, min_run_bits(dtype), r))
            return fail(TS_EINVAL, "internal: stage plan does not fit");
        for (int q = 0; q < (1 << RB); ++q) {
            r.load_off[q] = ts::deposit((uint64_t)q << r.load_win, sw.tile_mask);
            r.store_off[q] = ts::deposit((uint64_t)q << r.store_win, sw.tile_mask);
        }
        if (r.diag_win >= 0) {
            ts_status st = get_diag_table(c, T, RB, sw.tile_mask, a.d.axis, a.d.tau, a.d.qturn,
                                          r.diag_win, &r.dtab);
            if (st != TS_OK) return st;
        }
        r.n_tiles = 1ull << (n - T);
        r.reverse = (int32_t)(pe->reg_args.size() & 1);
        // strided tiles (every group but the low one) in rotated order, for states of at least
        // kTileRotBytes: smaller ones lose more of the alternating order's cache hits than they
        // gain (the N = 27 chain, 1 and 2 GiB: 1.6% and 2.5% slower rotated)
        const size_t bytes = ((size_t)1 << n) * (dtype == TS_C128 ? 16 : 8);
        r.rot = (sw.group > 0 && n - T > kTileRot && bytes >= kTileRotBytes) ? kTileRot : 0;
        pe->reg_args.push_back(r);
    }
    pe->reg_bits = RB;
    pe->prepared = true;
    return TS_OK;
}

// ------------------------------------------------------------------ light-cone sweeps

// Tables of one light-cone phase step: the terms of level `lv` (axis, tau, quarter turns)
// that the step applies -- fields and quarter turns of the spins in `own`, the bonds in
// `bonds` -- for the tile whose bit i holds spin tile_q[i], register window [w, w + RB).
// Bonds to a spin outside the tile become a field on its partner that depends on the
// outside spin's bit: those bits (their workgroup-index positions in `rank`) select the row.
ts_status get_cone_tab(ts_ctx *c, int T, int RB, int w, const std::vector<int> &tile_q,
                       const std::vector<int> &rank, int axis, double tau, int qturn, uint64_t own,
                       const std::vector<int> &bonds, const ConeTab **out)
{
    const int n = c->n;
    std::vector<int> kof(n, -1);
    for (int i = 0; i < T; ++i) kof[tile_q[i]] = i;
    const bool energy = axis >= 0 && axis < 3;
    std::vector<int> partners;  // outside spins of cross bonds, in first-seen order
    std::vector<double> Jt((size_t)T * T, 0.0);
    std::vector<double> hf(T, 0.0);
    struct Cross { int k, slot; double J; };
    std::vector<Cross> cross;
    for (int q = 0; q < n; ++q) {
        if (!((own >> q) & 1)) continue;
        if (kof[q] < 0) return fail(TS_EINVAL, "internal: light-cone term outside the tile");
        if (energy) hf[kof[q]] += c->h[q][axis];
    }
    for (int b : bonds) {
        const int p = c->bi[b], q = c->bj[b];
        const double J = energy ? c->J[b][axis] : 0.0;
        if (kof[p] >= 0 && kof[q] >= 0) {
            Jt[(size_t)std::min(kof[p], kof[q]) * T + std::max(kof[p], kof[q])] += J;
        } else if (kof[p] >= 0 || kof[q] >= 0) {
            const int in = kof[p] >= 0 ? p : q, ext = kof[p] >= 0 ? q : p;
            int slot = -1;
            for (size_t i = 0; i < partners.size(); ++i)
                if (partners[i] == ext) slot = (int)i;
            if (slot < 0) {
                slot = (int)partners.size();
                partners.push_back(ext);
            }
            cross.push_back({kof[in], slot, J});
        } else {
            return fail(TS_EINVAL, "internal: light-cone bond outside the tile");
        }
    }
    if ((int)partners.size() > tsk::kConeRowBits)
        return fail(TS_EINVAL, "internal: light-cone step couples too many outside spins");
    uint32_t qmask = 0;
    for (int q = 0; q < n; ++q)
        if ((own >> q) & 1) qmask |= 1u << kof[q];
    uint64_t tb;
    std::memcpy(&tb, &tau, sizeof tb);
    std::string key = std::to_string(T) + "/" + std::to_string(RB) + "/" + std::to_string(w) + "/" +
                      std::to_string(axis) + "/" + std::to_string(tb) + "/" + std::to_string(qturn & 3) + "/" +
                      std::to_string(qmask) + "|";
    for (int q : tile_q) key += std::to_string(q) + ",";
    key += "|";
    for (int b : bonds) key += std::to_string(b) + ",";
    key += "|";
    for (int p : partners) key += std::to_string(rank[p]) + ",";
    auto it = c->cone_tabs.find(key);
    if (it != c->cone_tabs.end()) {
        *out = it->second.get();
        return TS_OK;
    }
    auto J = [&](int a, int b) { return a < b ? Jt[(size_t)a * T + b] : Jt[(size_t)b * T + a]; };
    auto sp = [](uint32_t t, int k) { return ((t >> k) & 1) ? 0.5 : -0.5; };
    auto qt = [](int m) {
        static const ts::cplx q[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
        return q[m & 3];
    };
    auto ex = [&](double e) { return ts::cplx(std::cos(tau * e), -std::sin(tau * e)); };
    auto in_win = [&](int k) { return k >= w && k < w + RB; };
    // workgroup rows: the fields that bonds to outside spins put on tile bits
    const int nr = (int)partners.size();
    std::vector<ts::cplx> rows((size_t)(1u << nr) * (T + 1));
    uint32_t xmask = 0;
    for (const Cross &x : cross) xmask |= 1u << x.k;
    for (uint32_t r = 0; r < (1u << nr); ++r) {
        std::vector<double> g(T, 0.0);
        for (const Cross &x : cross) g[x.k] += x.J * (((r >> x.slot) & 1) ? 0.5 : -0.5);
        ts::cplx *row = &rows[(size_t)r * (T + 1)];
        double gw = 0.0;  // window bits: every one down, and the square that flips it up
        for (int k = 0; k < T; ++k) {
            if (!((xmask >> k) & 1)) row[1 + k] = ts::cplx(1.0, 0.0);
            else if (in_win(k)) row[1 + k] = ex(g[k]), gw += g[k];
            else row[1 + k] = ex(0.5 * g[k]);
        }
        row[0] = ex(-0.5 * gw);
    }
    // per-thread and window tables
    const int nthr = 1 << (T - RB);
    std::vector<ts::cplx> tab((size_t)nthr * (1 + RB) + (1u << RB));
    for (int tid = 0; tid < nthr; ++tid) {
        const uint32_t t0 = (tid & ((1u << w) - 1u)) | ((uint32_t)(tid >> w) << (w + RB));
        double e = 0.0;
        for (int k1 = 0; k1 < T; ++k1) {
            if (in_win(k1)) continue;
            e += hf[k1] * sp(t0, k1);
            for (int k2 = k1 + 1; k2 < T; ++k2)
                if (!in_win(k2)) e += J(k1, k2) * sp(t0, k1) * sp(t0, k2);
        }
        double hw = 0.0;
        for (int v = 0; v < RB; ++v) {
            double h = 0.0;
            for (int k = 0; k < T; ++k)
                if (!in_win(k)) h += J(k, w + v) * sp(t0, k);
            tab[(size_t)tid * (1 + RB) + 1 + v] = ex(h);
            hw += h;
        }
        tab[(size_t)tid * (1 + RB)] = qt(qturn * __builtin_popcount(t0 & qmask)) * ex(e - 0.5 * hw);
    }
    for (uint32_t r = 0; r < (1u << RB); ++r) {
        double e = 0.0;
        for (int v1 = 0; v1 < RB; ++v1) {
            e += hf[w + v1] * sp(r, v1);
            for (int v2 = v1 + 1; v2 < RB; ++v2) e += J(w + v1, w + v2) * sp(r, v1) * sp(r, v2);
        }
        tab[(size_t)nthr * (1 + RB) + r] = qt(qturn * __builtin_popcount((r << w) & qmask)) * ex(e);
    }
    auto ct = std::make_unique<ConeTab>();
    ct->xmask = xmask;
    for (int v = 0; v < RB; ++v) {
        bool dep = (xmask >> (w + v)) & 1;
        for (int k = 0; k < T && !dep; ++k) dep = !in_win(k) && J(k, w + v) != 0.0;
        if (dep) ct->cmask |= 1u << v;
    }
    ts_status st = alloc(ct->wgf, rows.size() * sizeof(ts::cplx));
    if (st != TS_OK) return st;
    st = alloc(ct->dtab, tab.size() * sizeof(ts::cplx));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(ct->wgf.p, rows.data(), rows.size() * sizeof(ts::cplx), hipMemcpyHostToDevice));
    TS_HIP(hipMemcpy(ct->dtab.p, tab.data(), tab.size() * sizeof(ts::cplx), hipMemcpyHostToDevice));
    ct->n_row_bits = nr;
    for (int i = 0; i < nr; ++i) ct->row_bit[i] = (int8_t)rank[partners[i]];
    *out = ct.get();
    c->cone_tabs.emplace(key, std::move(ct));
    return TS_OK;
}

// Runs of a tile-bit -> memory-bit map (consecutive tile bits on consecutive memory bits).
bool cone_runs(const std::vector<int> &pos, tsk::Run *runs, int32_t *nruns)
{
    int nr = 0;
    for (int i = 0; i < (int)pos.size();) {
        int e = i + 1;
        while (e < (int)pos.size() && pos[e] == pos[e - 1] + 1) ++e;
        if (nr >= tsk::kConeRuns) return false;
        runs[nr++] = tsk::Run{(int8_t)i, (int8_t)(e - i), (int8_t)pos[i], 0};
        i = e;
    }
    *nruns = nr;
    return true;
}

// Stage program of one light-cone sweep: butterfly ops are covered by register windows
// (greedy: stay in the current window while it holds bits still to rotate, else move to the
// window holding most of them), each phase step runs in the window current at that point.
// Loads use a window above the s low tile bits (their lanes carry memory bits 0..s-1); stores
// use window 0 when the sweep moves other spins to the low memory bits (tile bits RB..RB+s-1).
bool cone_stages(const ts::ConeSweep &sw, int T, int RB, int s, tsk::ConeArgs &a,
                 std::vector<int> &phase_win, int *transposes)
{
    const int n = (int)sw.tile_q.size();
    if (n != T) return false;
    std::vector<int> kof(64, -1);
    for (int i = 0; i < T; ++i) kof[sw.tile_q[i]] = i;
    auto tbits = [&](uint64_t spins) {
        uint32_t m = 0;
        for (int q = 0; q < 64; ++q)
            if ((spins >> q) & 1) m |= 1u << kof[q];
        return m;
    };
    auto wm = [&](int w) { return ((1u << RB) - 1u) << w; };
    bool low_kept = true;
    for (int i = 0; i < s; ++i) low_kept &= sw.store_pos[i] == i && sw.load_pos[i] == i;
    bool low_moved = RB >= s;
    for (int i = 0; i < s && low_moved; ++i) low_moved = sw.store_pos[RB + i] == i;
    for (int i = 0; i < s; ++i)
        if (sw.load_pos[i] != i) return false;
    if (!low_kept && !low_moved) return false;
    if (s > RB || T < 2 * RB) return false;
    // Window choice by dynamic programming over the operations: the state is the current
    // register window (any start 0..T-RB), a butterfly op is covered by a sequence of at
    // most three windows (each bit rotated in the first window of the sequence that holds
    // it), a phase step runs in the current window, and the cost is the number of window
    // changes (LDS transposes), including the one to the store window.
    const int NW = T - RB + 1;
    const int INF = 1 << 20;
    struct Seq { int len; int w[3]; };
    std::vector<Seq> seqs;
    // windows of the sequences: the aligned ones [0, RB), [RB, 2RB), [T-RB, T) (unaligned
    // windows saved a few transposes but no time on the GPU)
    const int wins[3] = {0, RB, T - RB};
    for (int a1 : wins) {
        seqs.push_back({1, {a1, 0, 0}});
        for (int a2 : wins) {
            if (a2 == a1) continue;
            seqs.push_back({2, {a1, a2, 0}});
            for (int a3 : wins)
                if (a3 != a2) seqs.push_back({3, {a1, a2, a3}});
        }
    }
    // masks of the windows of a sequence for one op (0: the sequence does not fit the op)
    auto split = [&](const Seq &q, uint32_t m, uint32_t *part) {
        uint32_t rem = m;
        for (int i = 0; i < q.len; ++i) {
            part[i] = rem & wm(q.w[i]);
            if (!part[i]) return false;   // a window without work is never useful
            rem &= ~part[i];
        }
        return rem == 0;
    };
    std::vector<int> bops;                 // op indices of the butterfly ops
    for (size_t oi = 0; oi < sw.ops.size(); ++oi)
        if (sw.ops[oi].kind == 0) bops.push_back((int)oi);
    const size_t nb = bops.size();
    // dp[i][w]: fewest transposes with window w current after butterfly op i-1
    std::vector<std::vector<int>> dp(nb + 1, std::vector<int>(NW, INF));
    std::vector<std::vector<std::pair<int, int>>> from(nb + 1, std::vector<std::pair<int, int>>(NW, {-1, -1}));
    for (int w : wins)
        if (w >= s) dp[0][w] = 0;                 // load window: lanes must carry the low bits
    for (size_t i = 0; i < nb; ++i) {
        const uint32_t m = tbits(sw.ops[bops[i]].spins);
        for (size_t qi = 0; qi < seqs.size(); ++qi) {
            const Seq &q = seqs[qi];
            uint32_t part[3];
            if (!split(q, m, part)) continue;
            const int last = q.w[q.len - 1];
            for (int w = 0; w < NW; ++w) {
                if (dp[i][w] >= INF) continue;
                const int c = dp[i][w] + (q.w[0] != w) + (q.len - 1);
                if (c < dp[i + 1][last]) {
                    dp[i + 1][last] = c;
                    from[i + 1][last] = {w, (int)qi};
                }
            }
        }
    }
    int best = -1, bestc = INF;
    for (int w = 0; w < NW; ++w) {
        if (dp[nb][w] >= INF) continue;
        const int c = dp[nb][w] + (low_kept ? (w >= s ? 0 : 1) : (w != 0 ? 1 : 0));
        if (c < bestc) {
            bestc = c;
            best = w;
        }
    }
    if (best < 0) return false;
    std::vector<int> chosen(nb), win_after(nb + 1);
    win_after[nb] = best;
    for (size_t i = nb; i > 0; --i) {
        chosen[i - 1] = from[i][win_after[i]].second;
        win_after[i - 1] = from[i][win_after[i]].first;
    }
    a.load_win = win_after[0];
    int cur = a.load_win, ns = 0, tr = 0;
    phase_win.assign(sw.phases.size(), -1);
    auto push = [&](int w, int op, uint32_t mask, int ph) {
        if (ns >= tsk::kConeStages) return false;
        if (w != cur) ++tr;
        a.st[ns++] = tsk::cone_code(w, op, mask, ph);
        cur = w;
        return true;
    };
    size_t bi = 0;
    for (size_t oi = 0; oi < sw.ops.size(); ++oi) {
        const ts::ConeOp &op = sw.ops[oi];
        if (op.kind == 1) {
            if (op.phase < 0 || op.phase >= tsk::kConePhases) return false;
            // join the butterfly stage just emitted in this window, if it has no phase yet
            const uint32_t last = ns > 0 ? a.st[ns - 1] : 0u;
            if (ns > 0 && (int)(last & 15u) == cur && !((last >> 4) & 1u)) {
                a.st[ns - 1] = last | (1u << 4) | ((uint32_t)(op.phase & 63) << 9);
            } else if (!push(cur, 1, 0, op.phase)) {
                return false;
            }
            phase_win[op.phase] = cur;
            continue;
        }
        const Seq &q = seqs[chosen[bi++]];
        uint32_t part[3];
        if (!split(q, tbits(op.spins), part)) return false;
        for (int i = 0; i < q.len; ++i)
            if (!push(q.w[i], 0, part[i] >> q.w[i], 0)) return false;
    }
    a.n_stages = ns;
    if (low_kept) a.store_win = cur >= s ? cur : T - RB;
    else a.store_win = 0;
    if (a.store_win != cur) ++tr;
    *transposes = tr;
    return true;
}

// Device arguments of every sweep of a light-cone plan (tables included), built once.
ts_status prepare_cone(ts_ctx *c, PlanEntry *pe, int dtype)
{
    if (pe->cone_prepared) return TS_OK;
    const ts::ConePlan &P = pe->cone_plan;
    const int n = c->n, T = P.T, RB = c->reg_bits[dtype];
    if (RB != 4) return fail(TS_EINVAL, "internal: light-cone sweeps need 16 amplitudes per thread");
    std::vector<tsk::ConeArgs> args(P.sweeps.size());
    pe->cone_phase_win.assign(P.sweeps.size(), {});
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    for (size_t k = 0; k < P.sweeps.size(); ++k) {
        const ts::ConeSweep &sw = P.sweeps[k];
        tsk::ConeArgs &a = args[k];
        std::memset(&a, 0, sizeof a);
        for (int i = 0; i < T; ++i)
            if (pos[sw.tile_q[i]] != sw.load_pos[i]) return fail(TS_EINVAL, "internal: light-cone layout");
        uint64_t tmask = 0;
        for (int i = 0; i < T; ++i) tmask |= 1ull << sw.load_pos[i];
        const uint64_t all = (1ull << n) - 1;
        std::vector<int> rank(n, -1);
        for (int q = 0; q < n; ++q)
            if (!((tmask >> pos[q]) & 1)) rank[q] = __builtin_popcountll(all & ~tmask & ((1ull << pos[q]) - 1));
        const auto orun = ts::deposit_runs(all & ~tmask);
        if (!cone_runs(sw.load_pos, a.load_runs, &a.n_load_runs) ||
            !cone_runs(sw.store_pos, a.store_runs, &a.n_store_runs) || orun.size() > (size_t)tsk::kConeRuns)
            return fail(TS_EINVAL, "internal: light-cone layout has too many bit runs");
        a.n_out_runs = (int32_t)orun.size();
        for (size_t i = 0; i < orun.size(); ++i)
            a.out_runs[i] = tsk::Run{(int8_t)orun[i].src, (int8_t)orun[i].len, (int8_t)orun[i].dst, 0};
        std::vector<int> pw;
        int tr = 0;
        if (sw.phases.size() > (size_t)tsk::kConePhases || !cone_stages(sw, T, RB, P.s, a, pw, &tr))
            return fail(TS_EINVAL, "internal: light-cone stage program does not fit");
        pe->cone_phase_win[k] = pw;
        for (int r = 0; r < (1 << RB); ++r) {
            uint64_t lo = 0, so = 0;
            for (int j = 0; j < RB; ++j)
                if ((r >> j) & 1) {
                    lo |= 1ull << sw.load_pos[a.load_win + j];
                    so |= 1ull << sw.store_pos[a.store_win + j];
                }
            a.load_off[r] = lo;
            a.store_off[r] = so;
        }
        a.n_phases = (int32_t)sw.phases.size();
        for (size_t p = 0; p < sw.phases.size(); ++p) {
            const ts::ConePhase &ph = sw.phases[p];
            const ts::DiagStep &d = P.chain.diags[ph.level];
            const ConeTab *tab;
            ts_status st = get_cone_tab(c, T, RB, pw[p], sw.tile_q, rank, d.axis, d.tau, d.qturn, ph.own,
                                        ph.bonds, &tab);
            if (st != TS_OK) return st;
            tsk::ConePhaseArgs &pa = a.ph[p];
            static const double r2 = 0.70710678118654752440;
            static const double cs[8] = {1, r2, 0, -r2, -1, -r2, 0, r2};
            static const double sn[8] = {0, r2, 1, r2, 0, -r2, -1, -r2};
            double mag = std::ldexp(1.0, -(ph.half_scale / 2));
            if (ph.half_scale & 1) mag *= r2;
            pa.kre = mag * cs[ph.eighths & 7];
            pa.kim = mag * sn[ph.eighths & 7];
            pa.wgf = static_cast<const double *>(tab->wgf.p);
            pa.dtab = static_cast<const double *>(tab->dtab.p);
            pa.n_row_bits = tab->n_row_bits;
            pa.xmask = tab->xmask;
            pa.cmask = tab->cmask;
            for (int i = 0; i < tab->n_row_bits; ++i) pa.row_bit[i] = tab->row_bit[i];
        }
        // each phase stage names the thread-table entries its step reads
        for (int i = 0; i < a.n_stages; ++i)
            if ((a.st[i] >> 4) & 1u) a.st[i] |= tsk::cone_th_need(a.ph[(a.st[i] >> 9) & 63u].cmask) << 15;
        for (int i = 0; i < T; ++i) pos[sw.tile_q[i]] = sw.store_pos[i];
    }
    for (int q = 0; q < n; ++q)
        if (pos[q] != q) return fail(TS_EINVAL, "internal: light-cone plan does not restore the layout");
    ts_status st = alloc(pe->cone_dev, args.size() * sizeof(tsk::ConeArgs));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(pe->cone_dev.p, args.data(), args.size() * sizeof(tsk::ConeArgs), hipMemcpyHostToDevice));
    pe->cone_host.swap(args);
    pe->cone_prepared = true;
    return TS_OK;
}

// Gradient terms of every sweep of an adjoint light-cone plan (prepare_cone first).  A phase
// step applies the terms of its level for some fields and bonds; after it, both vectors are
// in that level's frame and carry the butterflies' gain not yet paid back, 2^(e/2) with e =
// (spin-layers applied so far) - (sum of the half_scale of the steps applied so far), the same
// for every amplitude.  The gradient of a parameter theta of the term exp(-i tau theta f(b))
// then gains -2 tau / 2^e * sum_b f(b) Im(conj(lambda_b) psi_b) (tau: the inverse chain's),
// f = s_i for a field on spin i and s_i s_j for a bond, s = +-1/2.  *ok is false where the
// terms do not fit the kernel's limits (the caller keeps the ping-pong form).
ts_status prepare_cone_grad(ts_ctx *c, PlanEntry *pe, bool *ok)
{
    if (pe->cone_grad_prepared) {
        *ok = pe->cone_grad_ok;
        return TS_OK;
    }
    const ts::ConePlan &P = pe->cone_plan;
    const int n = c->n, T = P.T, RB = 4;
    const int np = n + (int)c->bi.size();
    if (pe->cone_phase_win.size() != P.sweeps.size())
        return fail(TS_EINVAL, "internal: light-cone gradient terms before the sweep arguments");
    std::vector<tsk::ConeGradArgs> args(P.sweeps.size());
    std::vector<int> slots_of_sweep(P.sweeps.size(), 0);
    std::vector<int> pos(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    const uint64_t all = (1ull << n) - 1;
    bool fits = true;
    int e = 0;
    for (size_t k = 0; k < P.sweeps.size(); ++k) {
        const ts::ConeSweep &sw = P.sweeps[k];
        tsk::ConeGradArgs &g = args[k];
        std::memset(&g, 0, sizeof g);
        std::vector<int> kof(n, -1);
        uint64_t tmask = 0;
        for (int i = 0; i < T; ++i) {
            kof[sw.tile_q[i]] = i;
            tmask |= 1ull << sw.load_pos[i];
        }
        // a spin outside the tile is a bit of the workgroup's tile index
        std::vector<int> rank(n, -1);
        for (int q = 0; q < n; ++q)
            if (!((tmask >> pos[q]) & 1)) rank[q] = __builtin_popcountll(all & ~tmask & ((1ull << pos[q]) - 1));
        std::vector<int> e_after(sw.phases.size(), 0);
        for (const ts::ConeOp &op : sw.ops) {
            if (op.kind == 0) {
                e += __builtin_popcountll(op.spins);
            } else {
                e -= sw.phases[op.phase].half_scale;
                e_after[op.phase] = e;
            }
        }
        std::map<int, int> slot;   // gradient column -> accumulator
        for (size_t p = 0; p < sw.phases.size(); ++p) {
            const ts::ConePhase &ph = sw.phases[p];
            const ts::DiagStep &d = P.chain.diags[ph.level];
            const int w = pe->cone_phase_win[k][p];
            struct Term { int m; uint32_t w0, w1; };
            std::vector<Term> pt;
            auto add = [&](int col, int q1, int q2) {
                int m = 0, nout = 0;
                uint32_t tmask = 0, wmask = 0;
                for (int q : {q1, q2}) {
                    if (q < 0) continue;
                    const int kb = kof[q];
                    if (kb >= w && kb < w + RB) {
                        m |= 1 << (kb - w);
                        continue;
                    }
                    ++nout;
                    if (kb >= 0) tmask |= 1u << kb;
                    else wmask |= 1u << rank[q];
                }
                auto it = slot.find(col);
                const int sl = it != slot.end() ? it->second : (slot[col] = (int)slot.size());
                if (sl >= tsk::kConeGradSlots) fits = false;
                pt.push_back({m, (uint32_t)(sl & 0xff) | ((uint32_t)nout << 8) | (tmask << 12), wmask});
            };
            if (d.axis <= 2 && w >= 0) {
                g.coef[p] = -2.0 * d.tau * std::ldexp(1.0, -e_after[p]);
                for (int q = 0; q < n; ++q)
                    if ((ph.own >> q) & 1) add(d.axis * np + q, q, -1);
                for (int b : ph.bonds) add(d.axis * np + n + b, c->bi[b], c->bj[b]);
            }
            std::stable_sort(pt.begin(), pt.end(), [](const Term &u, const Term &v) { return u.m < v.m; });
            if (pt.size() > (size_t)tsk::kConeGradTerms) {
                fits = false;
                break;
            }
            size_t i = 0;
            for (int m = 0; m <= (1 << RB); ++m) {
                g.start[p][m] = (int32_t)i;
                while (m < (1 << RB) && i < pt.size() && pt[i].m == m) ++i;
            }
            for (size_t t = 0; t < pt.size(); ++t) {
                g.term[p][0][t] = pt[t].w0;
                g.term[p][1][t] = pt[t].w1;
            }
        }
        if (slot.size() > (size_t)tsk::kConeGradSlots) fits = false;
        if (!fits) break;
        g.n_slots = (int32_t)slot.size();
        for (const auto &kv : slot) g.col[kv.second] = (int32_t)kv.first;
        slots_of_sweep[k] = g.n_slots;
        for (int i = 0; i < T; ++i) pos[sw.tile_q[i]] = sw.store_pos[i];
    }
    if (fits && e != 0) return fail(TS_EINVAL, "internal: light-cone plan leaves the butterflies' gain unpaid");
    if (fits) {
        ts_status st = alloc(pe->cone_grad_dev, args.size() * sizeof(tsk::ConeGradArgs));
        if (st != TS_OK) return st;
        TS_HIP(hipMemcpy(pe->cone_grad_dev.p, args.data(), args.size() * sizeof(tsk::ConeGradArgs),
                         hipMemcpyHostToDevice));
        pe->cone_grad_slots.swap(slots_of_sweep);
    }
    pe->cone_grad_ok = fits;
    pe->cone_grad_prepared = true;
    *ok = fits;
    return TS_OK;
}

ts_status ham_dev(ts_ctx *c);

// Energy table D_axis(b) of one axis for the energy-table sweep variant: 2^N doubles
// (complex128) or floats (complex64), built once per context by a kernel on the null stream.
ts_status get_etab(ts_ctx *c, int dtype, int axis, const void **out)
{
    DevBuf &t = c->etab[dtype][axis];
    if (!t.p) {
        ts_status st = ham_dev(c);
        if (st != TS_OK) return st;
        st = alloc(t, ((size_t)1 << c->n) * (dtype == TS_C128 ? sizeof(double) : sizeof(float)));
        if (st != TS_OK) return st;
        TS_HIP(tsk::launch_energy_table(dtype, t.p, c->n, static_cast<const double *>(c->ham_h.p),
                                        static_cast<const tsk::HamBond *>(c->ham_b.p), (int)c->bi.size(), axis,
                                        nullptr));
        TS_HIP(hipStreamSynchronize(nullptr));
    }
    *out = t.p;
    return TS_OK;
}

// The energy-table variant's arguments of a prepared plan: each phase step's table and the
// global offsets of the registers in its layout.  *ok is false where a phase argument
// tau * D could leave the range of the kernel's sin/cos (|tau| * max|D| >= 2^20); the plan
// then runs the factorised phase step.
ts_status prepare_etab(ts_ctx *c, PlanEntry *pe, int dtype, bool *ok)
{
    if (!pe->etab_prepared) {
        double emax[3] = {0.0, 0.0, 0.0};
        for (int q = 0; q < c->n; ++q)
            for (int a = 0; a < 3; ++a) emax[a] += 0.5 * std::fabs(c->h[q][a]);
        for (size_t k = 0; k < c->bi.size(); ++k)
            for (int a = 0; a < 3; ++a) emax[a] += 0.25 * std::fabs(c->J[k][a]);
        bool fits = true;
        for (const tsk::RegSweepArgs &r : pe->reg_args)
            if (r.diag_win >= 0 && r.d.axis >= 0 && r.d.axis < 3 && std::fabs(r.d.tau) * emax[r.d.axis] >= 1048576.0)
                fits = false;
        for (size_t k = 0; fits && k < pe->reg_args.size(); ++k) {
            tsk::RegSweepArgs &r = pe->reg_args[k];
            r.etab = nullptr;
            if (r.diag_win < 0) continue;
            for (int q = 0; q < (1 << pe->reg_bits); ++q)
                r.diag_off[q] = ts::deposit((uint64_t)q << r.diag_win, pe->plan.sweeps[k].tile_mask);
            if (r.d.axis >= 0 && r.d.axis < 3) {
                ts_status st = get_etab(c, dtype, r.d.axis, &r.etab);
                if (st != TS_OK) return st;
            }
        }
        pe->etab_ok = fits;
        pe->etab_prepared = true;
    }
    *ok = pe->etab_ok;
    return TS_OK;
}

// Launch sweep k of a tiled plan on every vector.
ts_status run_sweep(ts_ctx *c, PlanEntry *pe, size_t k, int dtype, void *const *psi, int n_psi,
                    hipStream_t stream)
{
    ts_status st = prepare_sweeps(c, pe, dtype);
    if (st != TS_OK) return st;
    const int T = pe->plan.tile_bits;
    // variant 4 runs its ping-pong plans (light-cone form not chosen) like 3 / 0
    const int var = c->sweep_variant[dtype] == 4 ? (dtype == TS_C128 ? 3 : 0) : c->sweep_variant[dtype];
    if (var == 5) {   // phase steps from the energy tables (else as variant 0)
        bool ok = false;
        st = prepare_etab(c, pe, dtype, &ok);
        if (st != TS_OK) return st;
        if (ok) {
            for (int v = 0; v < n_psi; ++v)
                TS_HIP(tsk::launch_sweep_etab(dtype, T, pe->reg_bits, psi[v], pe->reg_args[k], stream));
            return TS_OK;
        }
    }
    if (var == 1) {
        const uint32_t nblocks = (uint32_t)(1ull << (c->n - T));
        for (int v = 0; v < n_psi; ++v)
            TS_HIP(tsk::launch_sweep(dtype, T, psi[v], pe->lds_args[k], nblocks, stream));
        return TS_OK;
    }
    // the pipelined kernel exists only where two register sets fit; elsewhere the one-tile
    // kernel runs the same stages
    const bool pipe = var == 2 && valid_config(dtype, c->n, T, pe->reg_bits, 2);
    // variant 3: the half-LDS kernel (more workgroups per CU) for the sweeps on the top bit
    // group, whose tiles span the whole state and gain most from the extra occupancy
    const bool half = var == 3 && valid_config(dtype, c->n, T, pe->reg_bits, 3) &&
                      pe->plan.groups.size() > 1 &&
                      pe->plan.sweeps[k].group == (int)pe->plan.groups.size() - 1;
    auto one = [&](void *p, const tsk::RegSweepArgs &a) {
        return half ? tsk::launch_sweep_half(T, pe->reg_bits, p, a, stream)
                    : tsk::launch_sweep_reg(dtype, T, pe->reg_bits, p, a, stream);
    };
    if (!pipe && n_psi == 2) {  // both states of a pair (the adjoint's psi and lambda) in one launch
        tsk::RegSweepArgs a = pe->reg_args[k];
        a.psi2 = psi[1];
        TS_HIP(one(psi[0], a));
        return TS_OK;
    }
    for (int v = 0; v < n_psi; ++v) {
        if (pipe)
            TS_HIP(tsk::launch_sweep_pipe(dtype, T, pe->reg_bits, psi[v], pe->reg_args[k], stream));
        else
            TS_HIP(one(psi[v], pe->reg_args[k]));
    }
    return TS_OK;
}

// A plan repeats a few phase steps (the same axis, step, scalar and quarter turns) many
// times: their factors per amplitude are formed once per plan (one workgroup each) and the
// resident kernel then multiplies by them, with the same rounding as forming them in place.
// Only for states of at most 2^13 amplitudes (the factor kernel's tile is complex128).
ts_status resident_factors(ts_ctx *c, PlanEntry *pe, tsk::ResidentArgs *ra)
{
    const int n = c->n;
    if (n > 13 || !c->res_fac) return TS_OK;
    if (!pe->resident_fac_ops.p) {
        std::vector<tsk::ResidentOp> ops, uniq;
        std::vector<int> which;
        for (const auto &sw : pe->plan.sweeps) {
            tsk::ResidentOp op{};
            op.d = sw.diag >= 0 ? pe->diag_args[sw.diag] : tsk::DiagArgs{-1, 0, 0.0, 1.0, 0.0};
            op.post = sw.post_mask != 0;
            op.rec = -1;
            int k = -1;
            if (op.d.axis >= 0) {
                for (size_t u = 0; u < uniq.size() && k < 0; ++u) {
                    const tsk::DiagArgs &e = uniq[u].d;
                    if (e.axis == op.d.axis && e.qturn == op.d.qturn && e.tau == op.d.tau &&
                        e.kre == op.d.kre && e.kim == op.d.kim)
                        k = (int)u;
                }
                if (k < 0) {
                    k = (int)uniq.size();
                    uniq.push_back(op);
                }
            }
            ops.push_back(op);
            which.push_back(k);
        }
        if (uniq.empty()) return TS_OK;
        const size_t ne = (size_t)1 << n;
        ts_status st = alloc(pe->resident_fac, uniq.size() * ne * sizeof(double2));
        if (st != TS_OK) return st;
        st = alloc(pe->resident_uniq, uniq.size() * sizeof(tsk::ResidentOp));
        if (st != TS_OK) return st;
        TS_HIP(hipMemcpy(pe->resident_uniq.p, uniq.data(), uniq.size() * sizeof(tsk::ResidentOp),
                         hipMemcpyHostToDevice));
        tsk::ResidentArgs fa = *ra;
        fa.ops = static_cast<const tsk::ResidentOp *>(pe->resident_uniq.p);
        fa.n_ops = (int)uniq.size();
        double2 *fac = static_cast<double2 *>(pe->resident_fac.p);
        TS_HIP(tsk::launch_resident_factors(n < 8 ? 8 : n, fa, fac, nullptr));
        for (size_t i = 0; i < ops.size(); ++i)
            if (which[i] >= 0) ops[i].fac = fac + (size_t)which[i] * ne;
        st = alloc(pe->resident_fac_ops, ops.size() * sizeof(tsk::ResidentOp));
        if (st != TS_OK) return st;
        TS_HIP(hipMemcpy(pe->resident_fac_ops.p, ops.data(), ops.size() * sizeof(tsk::ResidentOp),
                         hipMemcpyHostToDevice));
    }
    ra->ops = static_cast<const tsk::ResidentOp *>(pe->resident_fac_ops.p);
    return TS_OK;
}

// Op list and energy tables of a resident plan (the state fits one tile: no outside bits,
// the workgroup factors are the fields, the thread tables hold every coupling).
ts_status resident_args(ts_ctx *c, PlanEntry *pe, tsk::ResidentArgs *ra)
{
    ts_status st = resident_ops(pe);
    if (st != TS_OK) return st;
    const int n = c->n, Tk = n < 8 ? 8 : n;
    std::array<EnergyTable *, 3> tab{};
    for (int a = 0; a < 3; ++a) {
        if (c->zero_axis[a]) continue;
        st = get_table(c, Tk, (1ull << n) - 1, a, &tab[a]);
        if (st != TS_OK) return st;
    }
    ra->ops = static_cast<const tsk::ResidentOp *>(pe->resident_ops.p);
    ra->n_ops = (int)pe->plan.sweeps.size();
    ra->n = n;
    for (int a = 0; a < 3; ++a) {
        ra->wg[a] = tab[a] ? static_cast<const double *>(tab[a]->wg.p) : nullptr;
        ra->jt[a] = tab[a] ? static_cast<const double *>(tab[a]->jt.p) : nullptr;
    }
    return resident_factors(c, pe, ra);
}

// Segments one recorded resident launch runs at most.
constexpr int64_t kResidentReps = 4096;

// A recorded evolution of one vector that fits one tile, as single launches: `nseg` segments
// of one cached plan each, with the observables (real kinds) recorded from LDS into
// rows[k * slots ...] after segment k.  Returns false in *ran (and does nothing) when the
// segment's plan is not resident.
ts_status run_resident_records(ts_ctx *c, int dtype, int T, int order, double dt, int64_t seg,
                               int64_t nseg, void *psi, const std::vector<tsk::ObsDev> &obs, int slots,
                               double *rows, hipStream_t s, bool *ran)
{
    *ran = false;
    PlanEntry *pe;
    ts_status st = build_plan(c, dtype, T, order, dt, seg, &pe);
    if (st != TS_OK) return st;
    if (!pe->plan.resident) return TS_OK;
    tsk::ResidentArgs ra{};
    st = resident_args(c, pe, &ra);
    if (st != TS_OK) return st;
    ra.psi[0] = psi;
    for (size_t k = 0; k < obs.size(); ++k) ra.obs[k] = obs[k];
    ra.n_obs = (int)obs.size();
    ra.slots = slots;
    for (int64_t k = 0; k < nseg; k += kResidentReps) {
        ra.n_rep = (int32_t)std::min(kResidentReps, nseg - k);
        ra.rec_rows = rows + (size_t)k * slots;
        TS_HIP(tsk::launch_resident(dtype, c->n < 8 ? 8 : c->n, ra, 1, s));
    }
    *ran = true;
    return TS_OK;
}

// fuse: observables (ts_evolve's device form) that the last light-cone sweep of their ket
// vector accumulates into c->cone_partials, column = position in *fuse; *fused is set when
// this plan did so (light-cone form), and left alone otherwise.
ts_status run_plan(ts_ctx *c, PlanEntry *pe, int dtype, void *const *psi, int n_psi,
                   hipStream_t stream, const std::vector<tsk::ObsDev> *fuse = nullptr, bool *fused = nullptr)
{
    const ts::Plan &P = pe->plan;
    const int n = c->n;
    if (P.resident) {
        tsk::ResidentArgs ra{};
        ts_status st = resident_args(c, pe, &ra);
        if (st != TS_OK) return st;
        for (int v = 0; v < n_psi; ++v) ra.psi[v] = psi[v];
        TS_HIP(tsk::launch_resident(dtype, n < 8 ? 8 : n, ra, n_psi, stream));
        return TS_OK;
    }
    if (pe->cone) {
        ts_status st = prepare_cone(c, pe, dtype);
        if (st != TS_OK) return st;
        const tsk::ConeArgs *dev = static_cast<const tsk::ConeArgs *>(pe->cone_dev.p);
        const uint64_t tiles = 1ull << (n - pe->cone_plan.T);
        if (fuse) {
            st = alloc(c->cone_partials, (size_t)tiles * 2 * tsk::kMaxObs * sizeof(double));
            if (st != TS_OK) return st;
        }
        const size_t last = pe->cone_plan.sweeps.size() - 1;
        for (int v = 0; v < n_psi; ++v) {
            tsk::ConeRec rec{};
            if (fuse)
                for (size_t g = 0; g < fuse->size(); ++g) {
                    const tsk::ObsDev &o = (*fuse)[g];
                    if (o.ket != v) continue;
                    rec.obs[rec.n_obs] = o;
                    rec.obs[rec.n_obs].slot = (int32_t)g;
                    rec.bra[rec.n_obs] = tsk::obs_complex(o.kind) ? psi[o.bra] : nullptr;
                    ++rec.n_obs;
                }
            rec.n = n;
            rec.partials = static_cast<double *>(c->cone_partials.p);
            for (size_t k = 0; k <= last; ++k) {
                if (k == last && rec.n_obs > 0)
                    TS_HIP(tsk::launch_cone_rec(dtype, pe->cone_plan.T, c->reg_bits[dtype], psi[v], dev + k,
                                                pe->cone_host[k].n_phases, tiles, (int)(k & 1), rec, stream));
                else
                    TS_HIP(tsk::launch_cone(dtype, pe->cone_plan.T, c->reg_bits[dtype], psi[v], dev + k,
                                            pe->cone_host[k].n_phases, tiles, (int)(k & 1), stream));
            }
        }
        if (fuse) c->cone_partial_rows = (int64_t)tiles;
        if (fused) *fused = fuse != nullptr;
        return TS_OK;
    }
    // one vector at a time: consecutive sweeps of one state alternate their tile order, so
    // the first tiles a sweep reads are the last the previous one wrote (still in cache)
    for (int v = 0; v < n_psi; ++v)
        for (size_t k = 0; k < P.sweeps.size(); ++k) {
            ts_status st = run_sweep(c, pe, k, dtype, psi + v, 1, stream);
            if (st != TS_OK) return st;
        }
    return TS_OK;
}

// Longest run one plan covers.  Longer runs repeat cached plans: host time and memory stay
// bounded, at the cost of one extra (low-group phase) sweep per chunk.
constexpr int64_t kChunkSteps = 32;

// fuse/fused: as for run_plan, applied to the last plan of the run.
ts_status run_steps(ts_ctx *c, int dtype, int T, int order, double dt, int64_t steps,
                    void *const *psi, int n_psi, hipStream_t s,
                    const std::vector<tsk::ObsDev> *fuse = nullptr, bool *fused = nullptr)
{
    while (steps > 0) {
        const int64_t k = std::min(steps, kChunkSteps);
        PlanEntry *pe;
        ts_status st = build_plan(c, dtype, T, order, dt, k, &pe);
        if (st != TS_OK) return st;
        const bool tail = steps == k;
        st = run_plan(c, pe, dtype, psi, n_psi, s, tail ? fuse : nullptr, tail ? fused : nullptr);
        if (st != TS_OK) return st;
        steps -= k;
    }
    return TS_OK;
}

// Validates the observables and writes their device form into dev[0..n_obs) (at most
// kMaxObs entries; no allocation).
ts_status check_obs(const ts_ctx *c, const ts_observable *obs, int n_obs, int n_psi, bool in_evolve,
                    tsk::ObsDev *dev, int *slots)
{
    if (n_obs < 0 || n_obs > tsk::kMaxObs) return fail(TS_EINVAL, "n_obs must be 0..16");
    if (n_obs > 0 && !obs) return fail(TS_EINVAL, "observables pointer is NULL");
    int s = 0;
    for (int k = 0; k < n_obs; ++k) {
        const ts_observable &o = obs[k];
        tsk::ObsDev d{};
        d.kind = o.kind;
        d.i = o.i;
        d.j = o.j;
        d.slot = s;
        switch (o.kind) {
        case TS_OBS_NORM: case TS_OBS_MZ: case TS_OBS_ENERGY: case TS_OBS_OVERLAP: break;
        case TS_OBS_SX: case TS_OBS_SY: case TS_OBS_SZ: case TS_OBS_OVERLAP_SZ:
            if (o.i < 0 || o.i >= c->n) return fail(TS_EINVAL, "observable spin index out of range");
            break;
        case TS_OBS_SZSZ:
            if (o.i < 0 || o.i >= c->n || o.j < 0 || o.j >= c->n)
                return fail(TS_EINVAL, "observable spin index out of range");
            break;
        default: return fail(TS_EINVAL, "unknown observable kind");
        }
        if (in_evolve) {
            if (o.ket < 0 || o.ket >= n_psi) return fail(TS_EINVAL, "observable ket index out of range");
            d.ket = o.ket;
            if (tsk::obs_complex(o.kind)) {
                if (o.bra < 0 || o.bra >= n_psi) return fail(TS_EINVAL, "observable bra index out of range");
                d.bra = o.bra;
            }
        } else {
            d.ket = 0;
            if (tsk::obs_complex(o.kind)) {
                if (!o.other) return fail(TS_EINVAL, "overlap observable needs `other`");
                d.bra = 1 + k;  // filled by the caller
            }
        }
        s += tsk::obs_complex(o.kind) ? 2 : 1;
        dev[k] = d;
    }
    *slots = s;
    return TS_OK;
}

ts_status check_obs(const ts_ctx *c, const ts_observable *obs, int n_obs, int n_psi, bool in_evolve,
                    std::vector<tsk::ObsDev> &dev, int *slots)
{
    tsk::ObsDev d[tsk::kMaxObs];
    ts_status st = check_obs(c, obs, n_obs, n_psi, in_evolve, d, slots);
    if (st != TS_OK) return st;
    dev.insert(dev.end(), d, d + n_obs);
    return TS_OK;
}

constexpr int kRedBlocks = tsk::kScratchBlocks;

// Device copy of the Hamiltonian (fields, merged bonds) for the energy observable.
ts_status ham_dev(ts_ctx *c)
{
    if (c->ham_h.p) return TS_OK;
    std::vector<double> hf((size_t)3 * c->n);
    for (int q = 0; q < c->n; ++q)
        for (int a = 0; a < 3; ++a) hf[(size_t)3 * q + a] = c->h[q][a];
    std::vector<tsk::HamBond> hb(c->bi.size());
    for (size_t k = 0; k < hb.size(); ++k)
        hb[k] = tsk::HamBond{c->bi[k], c->bj[k], c->J[k][0], c->J[k][1], c->J[k][2]};
    ts_status st = alloc(c->ham_b, std::max<size_t>(1, hb.size()) * sizeof(tsk::HamBond));
    if (st != TS_OK) return st;
    if (!hb.empty()) TS_HIP(hipMemcpy(c->ham_b.p, hb.data(), hb.size() * sizeof(tsk::HamBond), hipMemcpyHostToDevice));
    st = alloc(c->ham_h, hf.size() * sizeof(double));
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpy(c->ham_h.p, hf.data(), hf.size() * sizeof(double), hipMemcpyHostToDevice));
    return TS_OK;
}

ts_status reduce(ts_ctx *c, int dtype, const void *const *vecs, int nvec,
                 const std::vector<tsk::ObsDev> &obs, double *out, hipStream_t stream)
{
    tsk::ReduceArgs ra{};
    for (int v = 0; v < nvec; ++v) ra.psi[v] = vecs[v];
    for (size_t k = 0; k < obs.size(); ++k) ra.obs[k] = obs[k];
    ra.n_obs = (int)obs.size();
    ra.n = c->n;
    ts_status st;
    for (const auto &o : obs)
        if (o.kind == TS_OBS_ENERGY) {
            st = ham_dev(c);
            if (st != TS_OK) return st;
            ra.ham_h = static_cast<const double *>(c->ham_h.p);
            ra.ham_b = static_cast<const tsk::HamBond *>(c->ham_b.p);
            ra.ham_nb = (int)c->bi.size();
            break;
        }
    st = alloc(c->partials, (size_t)kRedBlocks * 2 * tsk::kMaxObs * sizeof(double));
    if (st != TS_OK) return st;
    const uint64_t dim = 1ull << c->n;
    uint64_t nb = dim / (256 * 4);
    if (nb < 1) nb = 1;
    if (nb > (uint64_t)kRedBlocks) nb = kRedBlocks;
    TS_HIP(tsk::launch_reduce(dtype, ra, static_cast<double *>(c->partials.p), (int)nb, out, stream));
    return TS_OK;
}

bool aligned(const void *p, int dtype) { return ((uintptr_t)p % (dtype == TS_C128 ? 16 : 8)) == 0; }

// ------------------------------------------------------------------ tuning cache
//
// The autotuner (ts_autotune) times candidate kernel configurations and stores the fastest
// per (GPU architecture, spins, dtype, order) in a JSON file:
//   {"entries": [{"arch": "gfx950", "n": 27, "dtype": 0, "order": 4, "tile_bits": 12,
//                 "reg_bits": 4, "variant": 0, "ms_per_step": 28.1}, ...]}
// The reader accepts exactly that shape; anything else reads as an empty cache, so a
// damaged file only causes re-tuning.

struct TuneEntry {
    std::string arch;
    int n = 0, dtype = 0, order = 0, tile_bits = 0, reg_bits = 0, variant = 0;
    double ms = 0.0;
};

std::string tune_cache_path()
{
    if (const char *p = std::getenv("TSSPIN_TUNE_CACHE")) return p;
    const char *home = std::getenv("HOME");
    return std::string(home ? home : ".") + "/.cache/tsspin/tune.json";
}

std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        (void)hipGetLastError();
        return "none";
    }
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

bool parse_entry(const std::string &obj, TuneEntry &e)
{
    int found = 0;
    size_t p = 0;
    while (true) {
        const size_t k0 = obj.find('"', p);
        if (k0 == std::string::npos) break;
        const size_t k1 = obj.find('"', k0 + 1);
        if (k1 == std::string::npos) return false;
        const std::string key = obj.substr(k0 + 1, k1 - k0 - 1);
        size_t c = obj.find(':', k1);
        if (c == std::string::npos) return false;
        ++c;
        while (c < obj.size() && std::isspace((unsigned char)obj[c])) ++c;
        if (c >= obj.size()) return false;
        if (obj[c] == '"') {
            const size_t v1 = obj.find('"', c + 1);
            if (v1 == std::string::npos) return false;
            if (key == "arch") {
                e.arch = obj.substr(c + 1, v1 - c - 1);
                found |= 1;
            }
            p = v1 + 1;
            continue;
        }
        char *end = nullptr;
        const double v = std::strtod(obj.c_str() + c, &end);
        if (end == obj.c_str() + c || !std::isfinite(v)) return false;
        p = (size_t)(end - obj.c_str());
        if (key == "n") { e.n = (int)v; found |= 2; }
        else if (key == "dtype") { e.dtype = (int)v; found |= 4; }
        else if (key == "order") { e.order = (int)v; found |= 8; }
        else if (key == "tile_bits") { e.tile_bits = (int)v; found |= 16; }
        else if (key == "reg_bits") { e.reg_bits = (int)v; found |= 32; }
        else if (key == "variant") { e.variant = (int)v; found |= 64; }
        else if (key == "ms_per_step") { e.ms = v; found |= 128; }
    }
    return found == 255;
}

std::vector<TuneEntry> read_tune_cache(const std::string &path)
{
    std::vector<TuneEntry> out;
    FILE *f = std::fopen(path.c_str(), "rb");
    if (!f) return out;
    std::string s;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0 && s.size() < (1u << 24)) s.append(buf, got);
    std::fclose(f);
    const size_t lb = s.find('[');
    if (s.find("\"entries\"") == std::string::npos || lb == std::string::npos) return out;
    size_t p = lb + 1;
    while (true) {
        const size_t o0 = s.find_first_of("{]", p);
        if (o0 == std::string::npos) return {};
        if (s[o0] == ']') break;
        const size_t o1 = s.find('}', o0);
        if (o1 == std::string::npos) return {};
        TuneEntry e;
        if (!parse_entry(s.substr(o0 + 1, o1 - o0 - 1), e)) return {};
        out.push_back(e);
        p = o1 + 1;
    }
    return out;
}

bool write_tune_cache(const std::string &path, const std::vector<TuneEntry> &es)
{
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        std::string dir = path.substr(0, slash), cur;
        for (size_t i = 0; i <= dir.size(); ++i) {
            if (i == dir.size() || dir[i] == '/') {
                if (!cur.empty()) (void)mkdir(cur.c_str(), 0755);
            }
            if (i < dir.size()) cur += dir[i];
        }
    }
    const std::string tmp = path + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return false;
    std::fprintf(f, "{\"entries\": [");
    for (size_t i = 0; i < es.size(); ++i) {
        const TuneEntry &e = es[i];
        std::fprintf(f,
                     "%s\n  {\"arch\": \"%s\", \"n\": %d, \"dtype\": %d, \"order\": %d, \"tile_bits\": %d, "
                     "\"reg_bits\": %d, \"variant\": %d, \"ms_per_step\": %.6g}",
                     i ? "," : "", e.arch.c_str(), e.n, e.dtype, e.order, e.tile_bits, e.reg_bits, e.variant, e.ms);
    }
    std::fprintf(f, "\n]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path.c_str()) == 0;
}

bool valid_config(int dtype, int n, int T, int RB, int variant)
{
    const int hi = dtype == TS_C128 ? 13 : 14;
    if (T < 8 || T > hi || (RB != 3 && RB != 4) || variant < 0 || variant > 5) return false;
    if (variant == 4) return RB == 4 && (T == 11 || T == 12) && n >= 1;
    if (variant == 5) return T <= 13 && n >= 1;
    if (variant == 3 && (dtype != TS_C128 || RB != 4 || T < 11 || T > 12)) return false;
    if (variant != 1 && RB == 3 && T > 13) return false;
    if (variant == 2 && (T < 10 || T > 13 || (T == 13 && (dtype == TS_C128 || RB == 4)))) return false;
    return n >= 1;
}

void apply_config(ts_ctx *c, int dtype, int T, int RB, int variant)
{
    c->tile_bits[dtype] = T;
    c->reg_bits[dtype] = RB;
    c->sweep_variant[dtype] = variant;
    for (auto &ch : c->chains) apply_config(ch.get(), dtype, T, RB, variant);
    c->programs.clear();
    c->program_order.clear();
}

// First use of a dtype: take the cached tuning for this GPU and size, if there is one.
void consult_tune_cache(ts_ctx *c, int dtype, int order)
{
    if (c->tune_checked[dtype] || c->user_config[dtype]) return;
    c->tune_checked[dtype] = true;
    if (std::getenv("TSSPIN_NO_TUNE_CACHE")) return;
    const std::string arch = device_arch();
    for (const TuneEntry &e : read_tune_cache(tune_cache_path()))
        if (e.arch == arch && e.n == c->n && e.dtype == dtype && e.order == order &&
            valid_config(dtype, c->n, e.tile_bits, e.reg_bits, e.variant)) {
            apply_config(c, dtype, e.tile_bits, e.reg_bits, e.variant);
            return;
        }
}

// One kernel launch of a batched evolution.
struct BatchLaunch {
    int kind = 0;                 // 0 resident, 1 batched sweep, 2 batched observables,
                                  // 3 batched light-cone sweep
    int T = 0, RB = 0;
    uint32_t count = 0;           // workgroups (resident) or chains
    tsk::ResidentArgs ra{};
    tsk::RegSweepArgs sa{};
    tsk::BatchReduceArgs ba{};
    double *partials = nullptr;
    int nbpc = 0;
    // kind 3: chain c's state at element cone_off[c] of cone_packed, its arguments cone_args[c]
    void *cone_packed = nullptr;
    const int64_t *cone_off = nullptr;
    const tsk::ConeArgs *cone_args = nullptr;
    uint64_t tiles = 0;
    int reverse = 0;
};

}  // namespace

// Everything one ts_evolve_batch call launches, with the device arrays it points to, its
// streams (one per class of chains of equal size, so the classes run concurrently) and the
// hipGraph captured from it.
struct BatchProgram {
    int dtype = 0;
    std::vector<std::vector<BatchLaunch>> per_class;
    std::vector<std::unique_ptr<DevBuf>> bufs;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;   // [0] fork, [1] entry from the caller, then one join per class
    hipStream_t cap = nullptr;        // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~BatchProgram()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t e : events) (void)hipEventDestroy(e);
        for (hipStream_t s : streams) (void)hipStreamDestroy(s);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

ts_ctx::~ts_ctx() = default;

namespace {

template <typename Tv>
ts_status upload(BatchProgram *bp, const std::vector<Tv> &v, const Tv **out)
{
    auto b = std::make_unique<DevBuf>();
    ts_status st = alloc(*b, std::max<size_t>(1, v.size()) * sizeof(Tv));
    if (st != TS_OK) return st;
    if (!v.empty()) TS_HIP(hipMemcpy(b->p, v.data(), v.size() * sizeof(Tv), hipMemcpyHostToDevice));
    *out = static_cast<const Tv *>(b->p);
    bp->bufs.push_back(std::move(b));
    return TS_OK;
}

hipError_t run_launch(int dtype, const BatchLaunch &L, hipStream_t s)
{
    switch (L.kind) {
    case 0: return tsk::launch_resident(dtype, L.T, L.ra, (int)L.count, s);
    case 1: return tsk::launch_sweep_reg_batch(dtype, L.T, L.RB, L.sa, L.count, s);
    case 3:
        return tsk::launch_cone_batch(dtype, L.T, L.RB, L.cone_packed, L.cone_off, L.cone_args, L.count, L.tiles,
                                      L.reverse, s);
    default: return tsk::launch_batch_reduce(dtype, L.ba, (int)L.count, L.partials, L.nbpc, s);
    }
}

// Build the launches of one batched evolution (all tables and device arrays are uploaded
// here, before any capture).
ts_status build_batch_program(ts_ctx *ctx, char *psi_packed, const int64_t *psi_off, int dtype,
                              double dt, int64_t nsteps, int order, const std::vector<tsk::ObsDev> &obs,
                              int slots, int rec_every, double *rec_out, BatchProgram *bp)
{
    const int nch = (int)ctx->chains.size();
    const size_t esz = dtype == TS_C128 ? 16 : 8;
    const bool rec = !obs.empty();
    const int64_t seg = rec ? rec_every : nsteps;
    const int64_t nseg = rec ? nsteps / seg : (nsteps > 0 ? 1 : 0);
    const int64_t rem = rec ? nsteps % seg : 0;
    const int64_t nrec = rec ? nsteps / rec_every + 1 : 0;
    const int Tdef = ctx->tile_bits[dtype] > 0 ? ctx->tile_bits[dtype] : default_tile_bits(dtype);
    bp->dtype = dtype;
    // classes: chains of equal size and equal vanishing axes share one plan
    std::map<int, std::vector<int>> classes;
    for (int c = 0; c < nch; ++c) {
        const ts_ctx *ch = ctx->chains[c].get();
        const int key = ch->n * 8 + ch->zero_axis[0] + 2 * ch->zero_axis[1] + 4 * ch->zero_axis[2];
        classes[key].push_back(c);
    }
    for (auto &kv : classes) {
        const std::vector<int> &mem = kv.second;
        ts_ctx *c0 = ctx->chains[mem[0]].get();
        const int n = c0->n;
        std::vector<BatchLaunch> L;
        PlanEntry *ps = nullptr, *pr = nullptr;
        ts_status st;
        if (nseg > 0) {
            st = build_plan(c0, dtype, Tdef, order, dt, seg, &ps);
            if (st != TS_OK) return st;
        }
        if (rem > 0) {
            st = build_plan(c0, dtype, Tdef, order, dt, rem, &pr);
            if (st != TS_OK) return st;
        }
        auto chain_psi = [&](int m) { return psi_packed + psi_off[m] * esz; };
        auto chain_rec = [&](int m) { return rec ? rec_out + (size_t)m * nrec * slots : nullptr; };
        if (n <= Tdef) {
            // LDS-resident: the whole evolution of every chain of the class in one launch
            const int Tk = n < 8 ? 8 : n;
            std::vector<tsk::ResidentOp> ops;
            auto add_plan = [&](PlanEntry *pe) {
                for (const auto &s : pe->plan.sweeps) {
                    tsk::ResidentOp op{};
                    op.d = s.diag >= 0 ? pe->diag_args[s.diag] : tsk::DiagArgs{-1, 0, 0.0, 1.0, 0.0};
                    op.post = s.post_mask != 0;
                    op.rec = -1;
                    ops.push_back(op);
                }
            };
            auto add_rec = [&](int r) {
                tsk::ResidentOp op{};
                op.d = tsk::DiagArgs{-1, 0, 0.0, 1.0, 0.0};
                op.post = 0;
                op.rec = r;
                ops.push_back(op);
            };
            if (rec) add_rec(0);
            for (int64_t k = 0; k < nseg; ++k) {
                add_plan(ps);
                if (rec) add_rec((int)(k + 1));
            }
            if (pr) add_plan(pr);
            std::vector<tsk::ResidentChain> rc;
            for (int m : mem) {
                ts_ctx *cm = ctx->chains[m].get();
                tsk::ResidentChain x{};
                x.psi = chain_psi(m);
                x.rec = chain_rec(m);
                for (int a = 0; a < 3; ++a) {
                    if (cm->zero_axis[a]) continue;
                    EnergyTable *t;
                    st = get_table(cm, Tk, (1ull << n) - 1, a, &t);
                    if (st != TS_OK) return st;
                    x.wg[a] = static_cast<const double *>(t->wg.p);
                    x.jt[a] = static_cast<const double *>(t->jt.p);
                }
                rc.push_back(x);
            }
            BatchLaunch bl;
            bl.kind = 0;
            bl.T = Tk;
            bl.count = (uint32_t)mem.size();
            st = upload(bp, ops, &bl.ra.ops);
            if (st != TS_OK) return st;
            st = upload(bp, rc, &bl.ra.chains);
            if (st != TS_OK) return st;
            bl.ra.n_ops = (int)ops.size();
            bl.ra.n = n;
            for (size_t o = 0; o < obs.size(); ++o) bl.ra.obs[o] = obs[o];
            bl.ra.n_obs = (int)obs.size();
            bl.ra.slots = slots;
            L.push_back(bl);
            bp->per_class.push_back(std::move(L));
            continue;
        }
        // tiled: one batched launch per sweep covers every chain of the class
        const int RB = c0->reg_bits[dtype];
        const uint64_t tiles = 1ull << (n - Tdef);
        auto sweep_arrays = [&](PlanEntry *pe_c0, int64_t steps, std::vector<const tsk::ChainPtrs *> &arr) {
            std::vector<PlanEntry *> pes;
            for (int m : mem) {
                PlanEntry *pe;
                ts_status s2 = build_plan(ctx->chains[m].get(), dtype, Tdef, order, dt, steps, &pe);
                if (s2 != TS_OK) return s2;
                s2 = prepare_sweeps(ctx->chains[m].get(), pe, dtype);
                if (s2 != TS_OK) return s2;
                pes.push_back(pe);
            }
            for (size_t k = 0; k < pe_c0->plan.sweeps.size(); ++k) {
                std::vector<tsk::ChainPtrs> cp;
                for (size_t q = 0; q < mem.size(); ++q) {
                    const tsk::RegSweepArgs &r = pes[q]->reg_args[k];
                    cp.push_back(tsk::ChainPtrs{chain_psi(mem[q]), r.wgf, r.dtab, chain_rec(mem[q])});
                }
                const tsk::ChainPtrs *p;
                ts_status s2 = upload(bp, cp, &p);
                if (s2 != TS_OK) return s2;
                arr.push_back(p);
            }
            return TS_OK;
        };
        // Light-cone form of the class where the cost model prefers it for its first chain
        // and every chain's plan has the same number of sweeps (one launch per sweep covers
        // all of them; each chain has its own stage programs and tables).
        bool cone = RB == 4 && (Tdef == 11 || Tdef == 12) && ctx->cone_mode != 0;
        std::vector<const tsk::ConeArgs *> cseg_arr, crem_arr;
        const int64_t *cone_off = nullptr;
        auto cone_arrays = [&](PlanEntry *pe_c0, int64_t steps, std::vector<const tsk::ConeArgs *> &arr) {
            PlanEntry probe;
            probe.plan = pe_c0->plan;
            if (!cone_candidate(c0, &probe, Tdef, dtype, ctx->cone_mode == 2 ? 2 : 1)) return false;
            std::vector<PlanEntry *> pes;
            for (int m : mem) {
                PlanEntry *pe;
                ts_ctx *cm = ctx->chains[m].get();
                if (build_plan(cm, dtype, Tdef, order, dt, steps, &pe) != TS_OK) return false;
                if (!pe->cone) pe->cone = cone_candidate(cm, pe, Tdef, dtype, 2);
                if (!pe->cone || pe->cone_plan.sweeps.size() != probe.cone_plan.sweeps.size()) return false;
                if (prepare_cone(cm, pe, dtype) != TS_OK) return false;
                pes.push_back(pe);
            }
            if (!cone_off) {
                std::vector<int64_t> off;
                for (int m : mem) off.push_back(psi_off[m]);
                if (upload(bp, off, &cone_off) != TS_OK) return false;
            }
            for (size_t k = 0; k < probe.cone_plan.sweeps.size(); ++k) {
                std::vector<tsk::ConeArgs> ca;
                for (size_t q = 0; q < mem.size(); ++q) ca.push_back(pes[q]->cone_host[k]);
                const tsk::ConeArgs *p;
                if (upload(bp, ca, &p) != TS_OK) return false;
                arr.push_back(p);
            }
            return true;
        };
        if (cone && ps) cone = cone_arrays(ps, seg, cseg_arr);
        if (cone && pr) cone = cone_arrays(pr, rem, crem_arr);
        (void)hipGetLastError();
        std::vector<const tsk::ChainPtrs *> seg_arr, rem_arr;
        if (ps && !cone) {
            st = sweep_arrays(ps, seg, seg_arr);
            if (st != TS_OK) return st;
        }
        if (pr && !cone) {
            st = sweep_arrays(pr, rem, rem_arr);
            if (st != TS_OK) return st;
        }
        BatchLaunch red;
        if (rec) {
            std::vector<tsk::ChainPtrs> cp;
            for (int m : mem) cp.push_back(tsk::ChainPtrs{chain_psi(m), nullptr, nullptr, chain_rec(m)});
            red.kind = 2;
            red.count = (uint32_t)mem.size();
            st = upload(bp, cp, &red.ba.chains);
            if (st != TS_OK) return st;
            for (size_t o = 0; o < obs.size(); ++o) red.ba.obs[o] = obs[o];
            red.ba.n_obs = (int)obs.size();
            red.ba.n = n;
            red.ba.slots = slots;
            uint64_t nbpc = (1ull << n) / 2048;
            red.nbpc = (int)std::max<uint64_t>(1, std::min<uint64_t>(64, nbpc));
            auto pb = std::make_unique<DevBuf>();
            st = alloc(*pb, mem.size() * red.nbpc * tsk::kMaxObs * sizeof(double));
            if (st != TS_OK) return st;
            red.partials = static_cast<double *>(pb->p);
            bp->bufs.push_back(std::move(pb));
        }
        auto add_cone = [&](const std::vector<const tsk::ConeArgs *> &arr) {
            for (size_t k = 0; k < arr.size(); ++k) {
                BatchLaunch bl;
                bl.kind = 3;
                bl.T = Tdef;
                bl.RB = 4;
                bl.count = (uint32_t)mem.size();
                bl.cone_packed = psi_packed;
                bl.cone_off = cone_off;
                bl.cone_args = arr[k];
                bl.tiles = tiles;
                bl.reverse = (int)(k & 1);
                L.push_back(bl);
            }
        };
        auto add_sweeps = [&](PlanEntry *pe_c0, const std::vector<const tsk::ChainPtrs *> &arr) {
            if (cone) {
                add_cone(pe_c0 == ps ? cseg_arr : crem_arr);
                return;
            }
            for (size_t k = 0; k < arr.size(); ++k) {
                BatchLaunch bl;
                bl.kind = 1;
                bl.T = Tdef;
                bl.RB = RB;
                bl.count = (uint32_t)mem.size();
                bl.sa = pe_c0->reg_args[k];
                bl.sa.chains = arr[k];
                bl.sa.tiles_per_chain = tiles;
                L.push_back(bl);
            }
        };
        if (ps && !cone) {
            st = prepare_sweeps(c0, ps, dtype);
            if (st != TS_OK) return st;
        }
        if (pr && !cone) {
            st = prepare_sweeps(c0, pr, dtype);
            if (st != TS_OK) return st;
        }
        if (rec) {
            red.ba.rec = 0;
            L.push_back(red);
        }
        for (int64_t k = 0; k < nseg; ++k) {
            add_sweeps(ps, seg_arr);
            if (rec) {
                red.ba.rec = (int)(k + 1);
                L.push_back(red);
            }
        }
        if (pr) add_sweeps(pr, rem_arr);
        bp->per_class.push_back(std::move(L));
    }
    return TS_OK;
}

// Capture the program into one graph: the caller's stream forks to one stream per class and
// joins back.  Returns false (and leaves no graph) if capture is not possible.
bool capture_batch_program(BatchProgram *bp)
{
    const size_t nc = bp->per_class.size();
    if (!bp->cap && hipStreamCreateWithFlags(&bp->cap, hipStreamNonBlocking) != hipSuccess) return false;
    while (bp->streams.size() < nc) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
        bp->streams.push_back(s);
    }
    while (bp->events.size() < nc + 2) {
        hipEvent_t e;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return false;
        bp->events.push_back(e);
    }
    if (hipStreamBeginCapture(bp->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    bool ok = hipEventRecord(bp->events[0], bp->cap) == hipSuccess;
    for (size_t c = 0; c < nc && ok; ++c) {
        ok = hipStreamWaitEvent(bp->streams[c], bp->events[0], 0) == hipSuccess;
        for (const BatchLaunch &L : bp->per_class[c]) {
            if (!ok) break;
            ok = run_launch(bp->dtype, L, bp->streams[c]) == hipSuccess;
        }
        ok = ok && hipEventRecord(bp->events[2 + c], bp->streams[c]) == hipSuccess;
        ok = ok && hipStreamWaitEvent(bp->cap, bp->events[2 + c], 0) == hipSuccess;
    }
    hipGraph_t g = nullptr;
    const bool ended = hipStreamEndCapture(bp->cap, &g) == hipSuccess;
    if (!ok || !ended || !g) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return false;
    }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return false;
    }
    bp->graph = g;
    bp->exec = ex;
    return true;
}

}  // namespace

extern "C" {

const char *ts_last_error(void) { return g_err.c_str(); }

ts_status ts_create(int32_t n_spins, const ts_bond *bonds, int32_t n_bonds, const double *fields,
                    ts_ctx **out)
{
    if (!out) return fail(TS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_spins < 1 || n_spins > kMaxSpinsC64)
        return fail(TS_EINVAL, "n_spins must be 1..35");
    if (n_bonds < 0) return fail(TS_EINVAL, "n_bonds < 0");
    if (n_bonds > 0 && !bonds) return fail(TS_EINVAL, "bonds is NULL");
    auto c = std::make_unique<ts_ctx>();
    c->n = n_spins;
    if (const char *v = std::getenv("TSSPIN_SWEEP_KERNEL")) {
        const int var = std::strcmp(v, "lds") == 0    ? 1
                        : std::strcmp(v, "pipe") == 0 ? 2
                        : std::strcmp(v, "half") == 0 ? 3
                        : std::strcmp(v, "cone") == 0 ? 4
                        : std::strcmp(v, "etab") == 0 ? 5
                                                      : 0;
        c->sweep_variant[TS_C128] = var;
        c->sweep_variant[TS_C64] = var == 3 ? 0 : var;   // the half-LDS kernel is complex128 only
    }
    if (const char *v = std::getenv("TSSPIN_REG_BITS")) {
        const int rb = std::atoi(v);
        if (rb == 3 || rb == 4) c->reg_bits[0] = c->reg_bits[1] = rb;
    }
    if (const char *v = std::getenv("TSSPIN_BALANCE")) c->balance = std::strcmp(v, "0") != 0;
    if (const char *v = std::getenv("TSSPIN_CONE")) c->cone_mode = std::atoi(v);
    if (const char *v = std::getenv("TSSPIN_CONE_ADV")) c->cone_adv = std::atoi(v);
    if (const char *v = std::getenv("TSSPIN_NO_FUSE")) c->no_fuse = std::strcmp(v, "0") != 0;
    if (const char *v = std::getenv("TSSPIN_RESIDENT_FACTORS")) c->res_fac = std::strcmp(v, "0") != 0;
    if (const char *v = std::getenv("TSSPIN_ADJ_SPLIT")) c->adj_split = std::strcmp(v, "0") != 0;
    if (const char *v = std::getenv("TSSPIN_ADJ_CONE")) c->adj_cone = std::strcmp(v, "0") != 0;
    c->h.assign(n_spins, {0.0, 0.0, 0.0});
    if (fields) {
        for (int j = 0; j < n_spins; ++j)
            for (int a = 0; a < 3; ++a) {
                const double v = fields[3 * j + a];
                if (!std::isfinite(v)) return fail(TS_EINVAL, "non-finite field");
                c->h[j][a] = v;
            }
    }
    std::map<std::pair<int, int>, size_t> seen;
    for (int k = 0; k < n_bonds; ++k) {
        const ts_bond &b = bonds[k];
        if (b.i < 0 || b.i >= n_spins || b.j < 0 || b.j >= n_spins)
            return fail(TS_EINVAL, "bond index out of range");
        if (b.i == b.j) return fail(TS_EINVAL, "bond with i == j");
        if (!std::isfinite(b.jx) || !std::isfinite(b.jy) || !std::isfinite(b.jz))
            return fail(TS_EINVAL, "non-finite coupling");
        const int p = b.i < b.j ? b.i : b.j, q = b.i < b.j ? b.j : b.i;
        auto key = std::make_pair(p, q);
        auto it = seen.find(key);
        if (it == seen.end()) {
            seen[key] = c->bi.size();
            c->input_bond.push_back((int)c->bi.size());
            c->bi.push_back(p);
            c->bj.push_back(q);
            c->J.push_back({b.jx, b.jy, b.jz});
        } else {
            c->input_bond.push_back((int)it->second);
            c->J[it->second][0] += b.jx;
            c->J[it->second][1] += b.jy;
            c->J[it->second][2] += b.jz;
        }
    }
    for (int a = 0; a < 3; ++a) {
        bool z = true;
        for (int j = 0; j < n_spins && z; ++j) z = c->h[j][a] == 0.0;
        for (size_t k = 0; k < c->J.size() && z; ++k) z = c->J[k][a] == 0.0;
        c->zero_axis[a] = z;
    }
    *out = c.release();
    return TS_OK;
}

ts_status ts_destroy(ts_ctx *ctx)
{
    if (!ctx) return TS_OK;
    if (ctx->device >= 0) (void)hipDeviceSynchronize();
    delete ctx;
    return TS_OK;
}

ts_status ts_evolve(ts_ctx *ctx, void *const *psi, int32_t n_psi, ts_dtype dtype, double dt,
                    int64_t nsteps, int32_t order, const ts_observable *rec, int32_t n_rec,
                    int32_t rec_every, double *rec_out, void *stream)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (ctx->n > (dtype == TS_C128 ? kMaxSpinsC128 : kMaxSpinsC64))
        return fail(TS_EINVAL, "too many spins for this dtype");
    if (n_psi < 1 || n_psi > tsk::kMaxVec) return fail(TS_EINVAL, "n_psi must be 1..8");
    if (!psi) return fail(TS_EINVAL, "psi is NULL");
    for (int v = 0; v < n_psi; ++v) {
        if (!psi[v]) return fail(TS_EINVAL, "psi[v] is NULL");
        if (!aligned(psi[v], dtype)) return fail(TS_EINVAL, "psi[v] is misaligned");
    }
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    if (nsteps < 0) return fail(TS_EINVAL, "nsteps < 0");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    std::vector<tsk::ObsDev> obs;
    int slots = 0;
    ts_status st = check_obs(ctx, rec, n_rec, n_psi, true, obs, &slots);
    if (st != TS_OK) return st;
    if (n_rec > 0) {
        if (rec_every < 1) return fail(TS_EINVAL, "rec_every must be >= 1");
        if (!rec_out) return fail(TS_EINVAL, "rec_out is NULL");
    }
    st = ensure_device(ctx);
    if (st != TS_OK) return st;
    consult_tune_cache(ctx, dtype, order);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const void *const *cpsi = const_cast<const void *const *>(psi);

    int64_t seg = n_rec > 0 ? rec_every : nsteps;
    int T = 0;
    st = resolve_tile(ctx, dtype, order, dt, std::max<int64_t>(1, std::min<int64_t>(seg, kChunkSteps)), &T);
    if (st != TS_OK) return st;
    int64_t nseg = (n_rec > 0 && seg > 0) ? nsteps / seg : (nsteps > 0 ? 1 : 0);
    int64_t rem = n_rec > 0 ? nsteps % seg : 0;
    std::vector<tsk::ObsDev> norms;
    if (ctx->watchdog >= 0.0) {
        for (int v = 0; v < n_psi; ++v) norms.push_back(tsk::ObsDev{TS_OBS_NORM, 0, 0, v, 0, v});
        st = alloc(ctx->watch_buf, 2 * tsk::kMaxVec * sizeof(double));
        if (st != TS_OK) return st;
        st = reduce(ctx, dtype, cpsi, n_psi, norms, static_cast<double *>(ctx->watch_buf.p), s);
        if (st != TS_OK) return st;
    }
    if (n_rec > 0) {
        st = reduce(ctx, dtype, cpsi, n_psi, obs, rec_out, s);
        if (st != TS_OK) return st;
    }
    // Observables that need only the amplitude at b (and a bra evolved before the ket) are
    // accumulated by the last light-cone sweep of their ket vector, when the segment runs in
    // that form; the rest (spin flips: S^x, S^y, the energy) by a reduction afterwards.
    std::vector<tsk::ObsDev> fuse, rest;
    int per_vec[tsk::kMaxVec] = {};
    for (const tsk::ObsDev &o : obs) {
        const bool diag = o.kind == TS_OBS_NORM || o.kind == TS_OBS_SZ || o.kind == TS_OBS_SZSZ ||
                          o.kind == TS_OBS_MZ || (tsk::obs_complex(o.kind) && o.bra < o.ket);
        const bool f = diag && !ctx->no_fuse && per_vec[o.ket] < tsk::kConeRecMax;
        if (f) ++per_vec[o.ket];
        (f ? fuse : rest).push_back(o);
    }
    // One vector that fits one tile, with observables the resident kernel can reduce (norm,
    // S^x, S^y, S^z, S^z S^z, M^z): every segment and record in one launch.
    int64_t first = 0;
    bool real_kinds = true;
    for (const tsk::ObsDev &o : obs) real_kinds = real_kinds && o.kind <= TS_OBS_MZ;
    if (n_rec > 0 && n_psi == 1 && nseg > 0 && seg <= kChunkSteps && real_kinds && !ctx->no_fuse) {
        bool ran = false;
        st = run_resident_records(ctx, dtype, T, order, dt, seg, nseg, psi[0], obs, slots, rec_out + slots, s,
                                  &ran);
        if (st != TS_OK) return st;
        if (ran) first = nseg;
    }
    for (int64_t k = first; k < nseg; ++k) {
        bool fused = false;
        st = run_steps(ctx, dtype, T, order, dt, seg, psi, n_psi, s, fuse.empty() ? nullptr : &fuse, &fused);
        if (st != TS_OK) return st;
        if (n_rec > 0) {
            double *row = rec_out + (size_t)(k + 1) * slots;
            if (fused) {
                tsk::ReduceArgs fa{};
                for (size_t g = 0; g < fuse.size(); ++g) fa.obs[g] = fuse[g];
                fa.n_obs = (int)fuse.size();
                fa.n = ctx->n;
                st = alloc(ctx->partials, (size_t)kRedBlocks * 2 * tsk::kMaxObs * sizeof(double));
                if (st != TS_OK) return st;
                TS_HIP(tsk::launch_finalize(static_cast<const double *>(ctx->cone_partials.p),
                                            (int)ctx->cone_partial_rows, fa, row,
                                            static_cast<double *>(ctx->partials.p), s));
                if (!rest.empty()) st = reduce(ctx, dtype, cpsi, n_psi, rest, row, s);
            } else {
                st = reduce(ctx, dtype, cpsi, n_psi, obs, row, s);
            }
            if (st != TS_OK) return st;
        }
    }
    if (rem > 0) {
        st = run_steps(ctx, dtype, T, order, dt, rem, psi, n_psi, s);
        if (st != TS_OK) return st;
    }
    if (!norms.empty()) {
        for (auto &o : norms) o.slot += n_psi;
        double *wb = static_cast<double *>(ctx->watch_buf.p);
        st = reduce(ctx, dtype, cpsi, n_psi, norms, wb, s);
        if (st != TS_OK) return st;
        double h[2 * tsk::kMaxVec];
        TS_HIP(hipMemcpyAsync(h, wb, 2 * n_psi * sizeof(double), hipMemcpyDeviceToHost, s));
        TS_HIP(hipStreamSynchronize(s));
        for (int v = 0; v < n_psi; ++v) {
            const double n0 = h[v], n1 = h[n_psi + v];
            if (!std::isfinite(n0) || !std::isfinite(n1) || std::fabs(n1 - n0) > ctx->watchdog * n0) {
                char msg[160];
                std::snprintf(msg, sizeof msg, "norm watchdog: vector %d norm %.17g -> %.17g (bound %.3g relative)",
                              v, n0, n1, ctx->watchdog);
                return fail(TS_ENUMERIC, msg);
            }
        }
    }
    return TS_OK;
}

ts_status ts_dt_bound(ts_ctx *ctx, double *bound)
{
    if (!ctx || !bound) return fail(TS_EINVAL, "ctx or bound is NULL");
    // Eq. SegundoMomento: the largest local second moment over spins j and their bond
    // partners k (k absent for a spin without bonds)
    auto field2 = [&](int j) {
        double f = 0.0;
        for (int a = 0; a < 3; ++a) f += 0.25 * ctx->h[j][a] * ctx->h[j][a];
        return f;
    };
    double worst = 0.0;
    for (int j = 0; j < ctx->n; ++j) worst = std::max(worst, field2(j));
    for (size_t k = 0; k < ctx->bi.size(); ++k) {
        double c = 0.0;
        for (int a = 0; a < 3; ++a) c += ctx->J[k][a] * ctx->J[k][a] / 16.0;
        worst = std::max(worst, std::max(field2(ctx->bi[k]), field2(ctx->bj[k])) + c);
    }
    *bound = worst > 0.0 ? 1.0 / std::sqrt(worst) : HUGE_VAL;
    return TS_OK;
}

ts_status ts_set_watchdog(ts_ctx *ctx, double max_drift)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (std::isnan(max_drift)) return fail(TS_EINVAL, "max_drift is NaN");
    ctx->watchdog = max_drift;
    return TS_OK;
}

ts_status ts_expect(ts_ctx *ctx, const void *psi, ts_dtype dtype, const ts_observable *obs,
                    int32_t n_obs, double *out_host, void *stream)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (!psi || !aligned(psi, dtype)) return fail(TS_EINVAL, "psi is NULL or misaligned");
    if (!out_host) return fail(TS_EINVAL, "out_host is NULL");
    std::vector<tsk::ObsDev> dev;
    int slots = 0;
    ts_status st = check_obs(ctx, obs, n_obs, 1, false, dev, &slots);
    if (st != TS_OK) return st;
    st = ensure_device(ctx);
    if (st != TS_OK) return st;
    std::vector<const void *> vecs{psi};
    for (int k = 0; k < n_obs; ++k) {
        if (tsk::obs_complex(obs[k].kind)) {
            if (!aligned(obs[k].other, dtype)) return fail(TS_EINVAL, "other is misaligned");
            dev[k].bra = (int)vecs.size();
            vecs.push_back(obs[k].other);
        }
    }
    if ((int)vecs.size() > tsk::kMaxVec) return fail(TS_EINVAL, "too many overlap observables");
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = alloc(ctx->expect_out, 2 * tsk::kMaxObs * sizeof(double));
    if (st != TS_OK) return st;
    if (n_obs == 0) return TS_OK;
    st = reduce(ctx, dtype, vecs.data(), (int)vecs.size(), dev, static_cast<double *>(ctx->expect_out.p), s);
    if (st != TS_OK) return st;
    TS_HIP(hipMemcpyAsync(out_host, ctx->expect_out.p, slots * sizeof(double), hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    return TS_OK;
}

ts_status ts_expect_noalloc(ts_ctx *ctx, const void *psi, ts_dtype dtype, const ts_observable *obs,
                            int32_t n_obs, double *out_dev, void *stream)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (!psi || !aligned(psi, dtype)) return fail(TS_EINVAL, "psi is NULL or misaligned");
    if (!out_dev) return fail(TS_EINVAL, "out_dev is NULL");
    tsk::ReduceArgs ra{};
    int slots = 0;
    ts_status st = check_obs(ctx, obs, n_obs, 1, false, ra.obs, &slots);
    if (st != TS_OK) return st;
    int nvec = 1;
    ra.psi[0] = psi;
    for (int k = 0; k < n_obs; ++k) {
        if (obs[k].kind == TS_OBS_ENERGY)
            return fail(TS_EUNSUPPORTED, "ts_expect_noalloc: the energy needs the context's device "
                                         "copy of H (use ts_expect)");
        if (tsk::obs_complex(obs[k].kind)) {
            if (!aligned(obs[k].other, dtype)) return fail(TS_EINVAL, "other is misaligned");
            if (nvec >= tsk::kMaxVec) return fail(TS_EINVAL, "too many overlap observables");
            ra.obs[k].bra = nvec;
            ra.psi[nvec++] = obs[k].other;
        }
    }
    st = ensure_device(ctx);
    if (st != TS_OK) return st;
    if (n_obs == 0) return TS_OK;
    ra.n_obs = n_obs;
    ra.n = ctx->n;
    uint64_t nb = (1ull << ctx->n) / (256 * 4);
    if (nb < 1) nb = 1;
    if (nb > (uint64_t)tsk::kScratchBlocks) nb = tsk::kScratchBlocks;
    if (nb * 2 * tsk::kMaxObs > tsk::kScratchDoubles)
        return fail(TS_EINVAL, "ts_expect_noalloc: the reduction needs more than the fixed scratch");
    double *scr = nullptr;
    TS_HIP(tsk::scratch_address(&scr));
    // every partial the finalize step reads is written by this call's reduction first
    TS_HIP(tsk::launch_reduce(dtype, ra, scr, (int)nb, out_dev, static_cast<hipStream_t>(stream)));
    return TS_OK;
}

ts_status ts_plan_describe(ts_ctx *ctx, ts_dtype dtype, double dt, int64_t nsteps, int32_t order,
                           int32_t tile_bits, int64_t *out, int64_t cap, int64_t *n_sweeps)
{
    if (!ctx || !n_sweeps) return fail(TS_EINVAL, "ctx or n_sweeps is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    if (nsteps < 1) return fail(TS_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    int T = tile_bits;
    if (T <= 0) {
        ts_status st = resolve_tile(ctx, dtype, order, dt, std::min<int64_t>(nsteps, kChunkSteps), &T);
        if (st != TS_OK) return st;
    }
    if (T < 2 || T > 20) return fail(TS_EINVAL, "tile_bits out of range");
    ts::Plan P;
    try {
        auto chain = ts::build_chain(order, dt, nsteps, ctx->zero_axis);
        P = ts::make_plan(chain, ctx->n, T, min_run_bits(dtype), false, ctx->balance);
    } catch (const std::exception &e) {
        return fail(TS_EINVAL, std::string("plan: ") + e.what());
    }
    *n_sweeps = (int64_t)P.sweeps.size();
    if (!out) return TS_OK;
    const int RB = ctx->reg_bits[dtype];
    for (int64_t k = 0; k < *n_sweeps && k < cap; ++k) {
        const ts::Sweep &s = P.sweeps[k];
        int64_t *r = out + 16 * k;
        r[0] = (int64_t)s.tile_mask;
        r[1] = (int64_t)s.pre_mask;
        r[2] = (int64_t)s.post_mask;
        if (s.diag >= 0) {
            const ts::DiagStep &d = P.chain.diags[s.diag];
            r[3] = d.axis;
            r[4] = d.qturn;
            r[5] = d.mag_exp;
            r[6] = d.mag_sqrt;
            r[7] = d.eighths;
            std::memcpy(&r[10], &d.tau, sizeof(double));
        } else {
            r[3] = -1;
            r[4] = r[5] = r[6] = r[7] = 0;
            r[10] = 0;
        }
        r[8] = P.tile_bits;
        r[9] = s.group;
        r[11] = 0;
        r[12] = r[13] = r[14] = r[15] = 0;
        if (P.resident) continue;
        tsk::RegSweepArgs ra{};
        if (!make_stages(P.tile_bits, RB, (uint32_t)to_tile_bits(s.pre_mask, s.tile_mask),
                         (uint32_t)to_tile_bits(s.post_mask, s.tile_mask), s.diag >= 0,
                         min_run_bits(dtype), ra))
            return fail(TS_EINVAL, "internal: stage plan does not fit");
        int transposes = 0, cur = ra.load_win;
        for (int st = 0; st < ra.n_stages; ++st) {
            const int w = (int)((ra.st_code[st / tsk::kStagesPerWord] >> (9 * (st % tsk::kStagesPerWord))) & 15u);
            transposes += w != cur;
            cur = w;
        }
        transposes += cur != ra.store_win;
        r[12] = RB;
        r[13] = (int64_t)ra.load_win | ((int64_t)ra.store_win << 8) | ((int64_t)(ra.diag_win + 1) << 16) |
                ((int64_t)ra.n_stages << 24) | ((int64_t)transposes << 32);
        r[14] = (int64_t)ra.st_code[0];
        r[15] = (int64_t)ra.st_code[1];
    }
    return TS_OK;
}

ts_status ts_cone_describe(ts_ctx *ctx, ts_dtype dtype, double dt, int64_t nsteps, int32_t order,
                           int32_t tile_bits, int32_t low_bits, int32_t max_adv, int64_t *out,
                           int64_t cap, int64_t *n_rows, int32_t *used)
{
    if (!ctx || !n_rows) return fail(TS_EINVAL, "ctx or n_rows is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    if (nsteps < 1) return fail(TS_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    // the light-cone form runs at the default width; ts_evolve takes it only where it also
    // keeps that width (resolve_tile)
    const int T = tile_bits > 0 ? tile_bits : default_tile_bits(dtype);
    int T_run = T;
    if (tile_bits <= 0) {
        ts_status st = resolve_tile(ctx, dtype, order, dt, std::min<int64_t>(nsteps, kChunkSteps), &T_run);
        if (st != TS_OK) return st;
    }
    const int s = low_bits > 0 ? low_bits : kConeLowBits;
    if (T < 2 || T > 20 || s >= T) return fail(TS_EINVAL, "tile_bits or low_bits out of range");
    ts::Plan P;
    ts::ConePlan cp;
    try {
        auto chain = ts::build_chain(order, dt, nsteps, ctx->zero_axis);
        P = ts::make_plan(chain, ctx->n, T, min_run_bits(dtype), false, ctx->balance);
    } catch (const std::exception &e) {
        return fail(TS_EINVAL, std::string("plan: ") + e.what());
    }
    std::vector<std::pair<int, int>> bonds;
    for (size_t k = 0; k < ctx->bi.size(); ++k) bonds.push_back({ctx->bi[k], ctx->bj[k]});
    if (!ts::make_cone_plan(P.chain, ctx->n, T, s, bonds, max_adv, 1u << 20, cp, tsk::kConePhases))
        return fail(TS_EINVAL, "no light-cone plan for these sizes");
    if (used) {
        *used = 0;
        const int cm = ctx->cone_mode >= 0 ? ctx->cone_mode : (ctx->sweep_variant[dtype] == 4 ? 1 : 0);
        if (cm > 0 && T_run == T && ctx->reg_bits[dtype] == 4 && !P.resident && valid_config(dtype, ctx->n, T, 4, 4)) {
            PlanEntry pe;
            pe.plan = P;
            *used = cone_candidate(ctx, &pe, T, dtype, cm) ? 1 : 0;
        }
    }
    int64_t k = 0;
    auto row = [&](std::initializer_list<int64_t> v) {
        if (out && k < cap) {
            int64_t *r = out + 10 * k;
            int i = 0;
            for (int64_t x : v) r[i++] = x;
            for (; i < 10; ++i) r[i] = 0;
        }
        ++k;
    };
    const int RB = ctx->reg_bits[dtype];
    for (const ts::ConeSweep &sw : cp.sweeps) {
        uint64_t win = 0, lo_l = 0, lo_s = 0;
        for (int i = 0; i < T; ++i) {
            win |= 1ull << sw.tile_q[i];
            if (sw.load_pos[i] < s) lo_l |= 1ull << sw.tile_q[i];
            if (sw.store_pos[i] < s) lo_s |= 1ull << sw.tile_q[i];
        }
        int64_t nst = 0, tr = 0, a_load = -1, a_store = -1;
        std::vector<int> pw(sw.phases.size(), -1);
        std::vector<uint32_t> prog;
        if (RB == 4 && T >= 8) {
            tsk::ConeArgs a;
            int t = 0;
            if (cone_stages(sw, T, RB, s, a, pw, &t)) {
                nst = a.n_stages;
                tr = t;
                a_load = a.load_win;
                a_store = a.store_win;
                prog.assign(a.st, a.st + a.n_stages);
            } else {
                nst = tr = -1;
            }
        }
        row({1, (int64_t)win, (int64_t)lo_l, (int64_t)lo_s, sw.remap ? 1 : 0, (int64_t)sw.ops.size(), nst, tr});
        for (int i = 0; i < T; ++i) row({4, i, sw.tile_q[i], sw.load_pos[i], sw.store_pos[i]});
        if (nst > 0) {
            row({5, -1, 0, 0, -1, a_load, 0, 0, 0, 0});
            for (int64_t i = 0; i < nst; ++i) {
                const uint32_t c = prog[i];
                row({5, (int64_t)(c & 15u), (int64_t)((c >> 4) & 1u), (int64_t)((c >> 5) & 15u),
                     (int64_t)((c >> 9) & 63u)});
            }
            row({5, -2, 0, 0, -1, a_store, 0, 0, 0, 0});
        }
        for (const ts::ConeOp &op : sw.ops) {
            if (op.kind == 0) {
                row({2, (int64_t)op.spins});
                continue;
            }
            const ts::ConePhase &ph = sw.phases[op.phase];
            const ts::DiagStep &d = cp.chain.diags[ph.level];
            int64_t bm = 0;
            if (bonds.size() <= 63) {
                for (int b : ph.bonds) bm |= 1ll << b;
            } else {
                bm = -1;
            }
            int64_t tb;
            std::memcpy(&tb, &d.tau, sizeof tb);
            row({3, ph.level, (int64_t)ph.own, bm, ph.half_scale, ph.eighths, d.axis, d.qturn, tb,
                 pw[op.phase]});
        }
    }
    *n_rows = k;
    return TS_OK;
}

}  // extern "C"

extern "C" ts_status ts_adjoint(ts_ctx *ctx, const void *psi0, ts_dtype dtype, double dt,
                                int64_t nsteps, int32_t order, const ts_observable *loss_obs,
                                double *loss, double *grad_bonds, double *grad_fields,
                                void *workspace, void *stream)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    const int n = ctx->n;
    if (n > (dtype == TS_C128 ? kMaxSpinsC128 : kMaxSpinsC64))
        return fail(TS_EINVAL, "too many spins for this dtype");
    if (!psi0 || !aligned(psi0, dtype)) return fail(TS_EINVAL, "psi0 is NULL or misaligned");
    if (!workspace || !aligned(workspace, dtype)) return fail(TS_EINVAL, "workspace is NULL or misaligned");
    if (!loss_obs || !loss || !grad_fields || (!grad_bonds && !ctx->input_bond.empty()))
        return fail(TS_EINVAL, "NULL loss, observable or gradient pointer");
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    if (nsteps < 0) return fail(TS_EINVAL, "nsteps < 0");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    const ts_observable &ob = *loss_obs;
    switch (ob.kind) {
    case TS_OBS_SX: case TS_OBS_SY: case TS_OBS_SZ:
        if (ob.i < 0 || ob.i >= n) return fail(TS_EINVAL, "observable spin index out of range");
        break;
    case TS_OBS_SZSZ:
        if (ob.i < 0 || ob.i >= n || ob.j < 0 || ob.j >= n)
            return fail(TS_EINVAL, "observable spin index out of range");
        break;
    case TS_OBS_MZ: case TS_OBS_ENERGY: break;
    default: return fail(TS_EINVAL, "loss observable must be SX, SY, SZ, SZSZ, MZ or ENERGY");
    }
    ts_status st = ensure_device(ctx);
    if (st != TS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t esz = dtype == TS_C128 ? 16 : 8;
    if (n < kAdjMinSpins) {
        // Below the smallest tile the kernels take, run the same problem on kAdjMinSpins
        // spins: the added spins have no field and no bond, so the state stays a product
        // with all of them down and every gradient of the original parameters is unchanged.
        if (!ctx->adj_pad) {
            std::vector<ts_bond> bonds;
            for (size_t k = 0; k < ctx->bi.size(); ++k)
                bonds.push_back(ts_bond{ctx->bi[k], ctx->bj[k], ctx->J[k][0], ctx->J[k][1], ctx->J[k][2]});
            std::vector<double> f((size_t)3 * kAdjMinSpins, 0.0);
            for (int q = 0; q < n; ++q)
                for (int a = 0; a < 3; ++a) f[(size_t)3 * q + a] = ctx->h[q][a];
            ts_ctx *pc = nullptr;
            st = ts_create(kAdjMinSpins, bonds.data(), (int32_t)bonds.size(), f.data(), &pc);
            if (st != TS_OK) return st;
            ctx->adj_pad.reset(pc);
        }
        const size_t pbytes = ((size_t)1 << kAdjMinSpins) * esz;
        st = alloc(ctx->adj_pad_buf, 3 * pbytes);
        if (st != TS_OK) return st;
        char *p0 = static_cast<char *>(ctx->adj_pad_buf.p);
        TS_HIP(hipMemsetAsync(p0, 0, pbytes, s));
        TS_HIP(hipMemcpyAsync(p0, psi0, ((size_t)1 << n) * esz, hipMemcpyDeviceToDevice, s));
        std::vector<double> gb((size_t)3 * std::max<size_t>(1, ctx->bi.size())), gf((size_t)3 * kAdjMinSpins);
        st = ts_adjoint(ctx->adj_pad.get(), p0, dtype, dt, nsteps, order, loss_obs, loss, gb.data(), gf.data(),
                        p0 + pbytes, stream);
        if (st != TS_OK) return st;
        // the added spins stay down: each adds -1/2 to the total magnetisation
        if (ob.kind == TS_OBS_MZ) *loss += 0.5 * (kAdjMinSpins - n);
        for (int q = 0; q < n; ++q)
            for (int a = 0; a < 3; ++a) grad_fields[3 * q + a] = gf[(size_t)3 * q + a];
        for (size_t k = 0; k < ctx->input_bond.size(); ++k)
            for (int a = 0; a < 3; ++a) grad_bonds[3 * k + a] = gb[(size_t)3 * ctx->input_bond[k] + a];
        return TS_OK;
    }
    consult_tune_cache(ctx, dtype, order);
    const int Tdef = ctx->tile_bits[dtype] > 0 ? ctx->tile_bits[dtype] : default_tile_bits(dtype);
    const int T = n < Tdef ? n : Tdef;
    const size_t bytes = ((size_t)1 << n) * esz;
    void *psi = workspace;
    void *lam = static_cast<char *>(workspace) + bytes;
    void *vecs[2] = {psi, lam};

    // forward: psi(T)
    TS_HIP(hipMemcpyAsync(psi, psi0, bytes, hipMemcpyDeviceToDevice, s));
    st = run_steps(ctx, dtype, Tdef, order, dt, nsteps, vecs, 1, s);
    if (st != TS_OK) return st;
    // loss and lambda = O psi(T)
    std::vector<tsk::ObsDev> od(1);
    od[0] = tsk::ObsDev{ob.kind, ob.i, ob.j, 0, 0, 0};
    st = alloc(ctx->expect_out, 2 * tsk::kMaxObs * sizeof(double));
    if (st != TS_OK) return st;
    const void *cv[1] = {psi};
    st = reduce(ctx, dtype, cv, 1, od, static_cast<double *>(ctx->expect_out.p), s);
    if (st != TS_OK) return st;
    const int P = n + (int)ctx->bi.size();
    if (ob.kind == TS_OBS_ENERGY) {
        // H itself depends on the parameters: the product rule adds <psi(T)|dH/dtheta|psi(T)>,
        // the spin operator (or product of two) that theta multiplies in Eq. 1
        st = alloc(ctx->grad_explicit, (size_t)3 * P * sizeof(double));
        if (st != TS_OK) return st;
        std::vector<tsk::ObsDev> terms;
        for (int a = 0; a < 3; ++a)
            for (int q = 0; q < P; ++q) {
                const int kind = q < n ? (a == 0 ? TS_OBS_SX : a == 1 ? TS_OBS_SY : TS_OBS_SZ)
                                       : (a == 0 ? tsk::kObsSxSx : a == 1 ? tsk::kObsSySy : TS_OBS_SZSZ);
                const int i = q < n ? q : ctx->bi[q - n], j = q < n ? 0 : ctx->bj[q - n];
                terms.push_back(tsk::ObsDev{kind, i, j, 0, 0, a * P + q});
                if ((int)terms.size() == tsk::kMaxObs) {
                    st = reduce(ctx, dtype, cv, 1, terms, static_cast<double *>(ctx->grad_explicit.p), s);
                    if (st != TS_OK) return st;
                    terms.clear();
                }
            }
        if (!terms.empty()) {
            st = reduce(ctx, dtype, cv, 1, terms, static_cast<double *>(ctx->grad_explicit.p), s);
            if (st != TS_OK) return st;
        }
        st = ham_dev(ctx);
        if (st != TS_OK) return st;
        TS_HIP(tsk::launch_apply_ham(dtype, psi, lam, n, static_cast<const double *>(ctx->ham_h.p),
                                     static_cast<const tsk::HamBond *>(ctx->ham_b.p), (int)ctx->bi.size(), s));
    } else {
        TS_HIP(tsk::launch_apply_obs(dtype, psi, lam, ob.kind, ob.i, ob.j, n, s));
    }

    // reverse: the chain for -dt undoes the forward one exactly; after each phase step
    // both vectors are in that step's frame and the gradient terms are accumulated
    // parameters: fields of every spin, then every merged bond, for each axis; workgroup b of
    // the gradient passes owns row b of the slots for the whole reverse pass.
    //  - light-cone pair sweeps (default where the inverse chain has a light-cone form that
    //    fits the kernel): psi and lambda through the light-cone stage programs in the same
    //    workgroup, the gradient sums of each phase step's own terms taken in registers
    //    (cone_pair kernels); one row per workgroup;
    //  - pair sweeps (otherwise): the reverse plan without split phases, each sweep on psi and
    //    lambda in the same workgroup, the gradient sums taken in registers after each phase
    //    step (sweep_pair_kernel); one row per tile;
    //  - otherwise (TSSPIN_ADJ_SPLIT, or a tile width or register window the pair kernel
    //    lacks) the split-phase plan with a separate pass per phase step: from 10 spins one
    //    pass for every parameter of the axis (grad_walsh_kernel, one wave per 2^10
    //    amplitudes), below chunks of kGradChunk parameters per pass.
    const bool pair = !ctx->adj_split && ctx->reg_bits[dtype] == 4 && T >= 8 && T <= 12;
    const bool cone_pair = pair && ctx->adj_cone && ctx->cone_mode != 0 && (T == 11 || T == 12) && n > T;
    const bool walsh = !pair && n >= 10;
    uint64_t nb = ((uint64_t)1 << n) / (256 * 4);
    if (nb < 1) nb = 1;
    if (nb > (uint64_t)kRedBlocks) nb = kRedBlocks;
    if (walsh) nb = (uint64_t)1 << (n - 10);
    if (pair) nb = (uint64_t)1 << (n - T);
    tsk::GradWalshArgs wa{};
    {
        // parameters grouped by the set of their spins among the index bits that vary along
        // a lane's amplitudes in the Walsh pass (the pair sweeps take them in any order)
        std::vector<int16_t> gi, gj, gc;
        constexpr int L = tsk::kGradWalshLow;
        auto in = [&](int q) { return q >= L && q < L + 4 ? 1 << (q - L) : 0; };
        for (int m = 0; m < 16; ++m) {
            wa.group_start[m] = (int32_t)gi.size();
            for (int q = 0; q < P; ++q) {
                const int i = q < n ? q : ctx->bi[q - n], j = q < n ? -1 : ctx->bj[q - n];
                const int low = in(i) | (j >= 0 ? in(j) : 0);
                if (low != m) continue;
                gi.push_back((int16_t)i);
                gj.push_back((int16_t)j);
                gc.push_back((int16_t)q);
            }
        }
        wa.group_start[16] = (int32_t)gi.size();
        if (!ctx->grad_params.p) {
            st = alloc(ctx->grad_params, 3 * gi.size() * sizeof(int16_t));
            if (st != TS_OK) return st;
            std::vector<int16_t> all(gi);
            all.insert(all.end(), gj.begin(), gj.end());
            all.insert(all.end(), gc.begin(), gc.end());
            TS_HIP(hipMemcpy(ctx->grad_params.p, all.data(), all.size() * sizeof(int16_t), hipMemcpyHostToDevice));
        }
        const int16_t *gp = static_cast<const int16_t *>(ctx->grad_params.p);
        wa.pi = gp;
        wa.pj = gp + P;
        wa.col = gp + 2 * P;
        wa.np = P;
        wa.n = n;
        wa.stride = 3 * P;
    }
    st = alloc(ctx->grad_acc, (size_t)3 * P * sizeof(double));
    if (st != TS_OK) return st;
    st = alloc(ctx->grad_slots, (size_t)nb * 3 * P * sizeof(double));
    if (st != TS_OK) return st;
    double *slots = static_cast<double *>(ctx->grad_slots.p);
    wa.slots = slots;
    TS_HIP(hipMemsetAsync(slots, 0, (size_t)nb * 3 * P * sizeof(double), s));
    std::vector<tsk::GradArgs> chunks;
    for (int p0 = 0; !pair && !walsh && p0 < P; p0 += tsk::kGradChunk) {
        tsk::GradArgs ga{};
        ga.np = std::min(tsk::kGradChunk, P - p0);
        ga.n = n;
        ga.slots = slots;
        ga.stride = 3 * P;
        ga.off = p0;
        for (int p = 0; p < ga.np; ++p) {
            const int q = p0 + p;
            ga.pi[p] = (int16_t)(q < n ? q : ctx->bi[q - n]);
            ga.pj[p] = (int16_t)(q < n ? -1 : ctx->bj[q - n]);
        }
        chunks.push_back(ga);
    }
    // the forward run was chunks of kChunkSteps steps and a shorter last one: undo them
    // last chunk first
    for (int64_t left = nsteps; left > 0;) {
        const int64_t chunk = (left % kChunkSteps) ? left % kChunkSteps : kChunkSteps;
        left -= chunk;
        PlanEntry *pr;
        st = build_plan(ctx, dtype, T, order, dt, chunk, &pr, true, !pair);
        if (st != TS_OK) return st;
        bool use_cone = false;
        if (cone_pair) {
            if (!pr->cone_tried) {
                pr->cone = cone_candidate(ctx, pr, T, dtype, 2);
                pr->cone_tried = true;
            }
            if (pr->cone) {
                st = prepare_cone(ctx, pr, dtype);
                if (st != TS_OK) return st;
                st = prepare_cone_grad(ctx, pr, &use_cone);
                if (st != TS_OK) return st;
            }
        }
        if (use_cone) {
            const tsk::ConeArgs *dev = static_cast<const tsk::ConeArgs *>(pr->cone_dev.p);
            const tsk::ConeGradArgs *gdev = static_cast<const tsk::ConeGradArgs *>(pr->cone_grad_dev.p);
            const uint64_t tiles = 1ull << (n - pr->cone_plan.T);
            for (size_t k = 0; k < pr->cone_plan.sweeps.size(); ++k)
                TS_HIP(tsk::launch_cone_pair(dtype, pr->cone_plan.T, 4, psi, lam, dev + k,
                                             pr->cone_host[k].n_phases, gdev + k, pr->cone_grad_slots[k],
                                             slots, 3 * P, tiles, (int)(k & 1), s));
            continue;
        }
        if (pair) {
            st = prepare_sweeps(ctx, pr, dtype);
            if (st != TS_OK) return st;
        }
        for (size_t k = 0; k < pr->plan.sweeps.size(); ++k) {
            const int di = pr->plan.sweeps[k].diag;
            const ts::DiagStep *d = di >= 0 ? &pr->plan.chain.diags[di] : nullptr;
            // the step applies exp(+i tau_fwd D) with tau = -tau_fwd; the states in its frame
            // carry a common scale 2^(carry/2)
            const double coef = d ? -2.0 * d->tau / (d->carry ? 2.0 : 1.0) : 0.0;
            if (pair) {
                tsk::PairGradArgs g{};
                g.pi = wa.pi;
                g.pj = wa.pj;
                g.col = wa.col;
                g.np = d && d->axis <= 2 ? P : 0;
                g.coef = coef;
                g.slots = slots;
                g.stride = 3 * P;
                g.off = d && d->axis <= 2 ? d->axis * P : 0;
                const uint64_t tm = pr->plan.sweeps[k].tile_mask;
                for (int q = 0; q < 64; ++q)
                    g.tile_bit[q] = (q < n && ((tm >> q) & 1)) ? (int8_t)__builtin_popcountll(tm & ((1ull << q) - 1))
                                                               : (int8_t)-1;
                TS_HIP(tsk::launch_sweep_pair(dtype, T, 4, psi, lam, pr->reg_args[k], g, s));
                continue;
            }
            st = run_sweep(ctx, pr, k, dtype, vecs, 2, s);
            if (st != TS_OK) return st;
            if (!d || d->axis > 2) continue;
            if (walsh) {
                tsk::GradWalshArgs w = wa;
                w.coef = coef;
                w.off = d->axis * P;
                TS_HIP(tsk::launch_grad_walsh(dtype, psi, lam, w, s));
                continue;
            }
            for (tsk::GradArgs ga : chunks) {
                ga.coef = coef;
                ga.off += d->axis * P;
                TS_HIP(tsk::launch_grad_reduce(dtype, psi, lam, ga, (int)nb, s));
            }
        }
    }
    TS_HIP(tsk::launch_grad_finalize(slots, (int)nb, 3 * P, static_cast<double *>(ctx->grad_acc.p), s));
    std::vector<double> g((size_t)3 * P), gx;
    TS_HIP(hipMemcpyAsync(g.data(), ctx->grad_acc.p, g.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    if (ob.kind == TS_OBS_ENERGY) {
        gx.resize(g.size());
        TS_HIP(hipMemcpyAsync(gx.data(), ctx->grad_explicit.p, gx.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    }
    TS_HIP(hipMemcpyAsync(loss, ctx->expect_out.p, sizeof(double), hipMemcpyDeviceToHost, s));
    TS_HIP(hipStreamSynchronize(s));
    for (size_t k = 0; k < gx.size(); ++k) g[k] += gx[k];
    for (int j = 0; j < n; ++j)
        for (int a = 0; a < 3; ++a) grad_fields[3 * j + a] = g[(size_t)a * P + j];
    for (size_t k = 0; k < ctx->input_bond.size(); ++k)
        for (int a = 0; a < 3; ++a) grad_bonds[3 * k + a] = g[(size_t)a * P + n + ctx->input_bond[k]];
    return TS_OK;
}

extern "C" ts_status ts_set_tile_bits(ts_ctx *ctx, ts_dtype dtype, int32_t tile_bits)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    const int hi = dtype == TS_C128 ? 13 : 14;
    if (tile_bits != 0 && (tile_bits < 8 || tile_bits > hi))
        return fail(TS_EINVAL, "tile_bits must be 0 or 8..13 (c128) / 8..14 (c64)");
    ctx->tile_bits[dtype] = tile_bits;
    ctx->user_config[dtype] = tile_bits != 0;
    for (auto &ch : ctx->chains) {
        ch->tile_bits[dtype] = tile_bits;
        ch->user_config[dtype] = tile_bits != 0;
    }
    ctx->programs.clear();
    ctx->program_order.clear();
    return TS_OK;
}

extern "C" ts_status ts_get_kernel_config(ts_ctx *ctx, ts_dtype dtype, int32_t order, int32_t *tile_bits,
                                          int32_t *reg_bits, int32_t *variant)
{
    if (!ctx || !tile_bits || !reg_bits || !variant) return fail(TS_EINVAL, "NULL argument");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    consult_tune_cache(ctx, dtype, order);
    int T = 0;
    ts_status st = resolve_tile(ctx, dtype, order, 1.0, 1, &T);   // the plan's shape does not depend on dt
    if (st != TS_OK) return st;
    *tile_bits = T;
    *reg_bits = ctx->reg_bits[dtype];
    *variant = ctx->sweep_variant[dtype];
    return TS_OK;
}

// Batch contexts: time one step of the whole batch (every size class, as one graph replay)
// for each tile width and register window; the best is kept on the context only.
static ts_status autotune_batch(ts_ctx *ctx, int dtype, int order, void *scratch, double *ms_per_step,
                         hipStream_t s)
{
    std::vector<int64_t> off(ctx->chains.size());
    int64_t total = 0;
    for (size_t c = 0; c < ctx->chains.size(); ++c) {
        off[c] = total;
        total += (int64_t)1 << ctx->chains[c]->n;
    }
    const int hi = dtype == TS_C128 ? 13 : 14;
    hipEvent_t e0, e1;
    TS_HIP(hipEventCreate(&e0));
    TS_HIP(hipEventCreate(&e1));
    double best = 1e300;
    int bT = 0, bRB = 0, bcone = 0;
    ts_status st = TS_OK;
    const int cone0 = ctx->cone_mode;
    for (int T = 8; T <= hi && st == TS_OK; ++T)
        for (int RB = 3; RB <= 4 && st == TS_OK; ++RB)
        for (int cone = 0; cone <= ((RB == 4 && (T == 11 || T == 12)) ? 1 : 0) && st == TS_OK; ++cone) {
            if (!valid_config(dtype, 1, T, RB, 0)) continue;
            apply_config(ctx, dtype, T, RB, 0);
            ctx->cone_mode = cone;   // light-cone classes where the cost model prefers them
            // first call builds and captures the program, the second replays it (timed)
            for (int rep = 0; rep < 2 && st == TS_OK; ++rep) {
                if (rep) (void)hipEventRecord(e0, s);
                st = ts_evolve_batch(ctx, scratch, off.data(), (ts_dtype)dtype, 0.01, 1, order, nullptr, 0, 1,
                                     nullptr, s);
                if (rep) (void)hipEventRecord(e1, s);
            }
            float ms = 0.f;
            if (st != TS_OK) break;
            if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(TS_EDEVICE, "timing failed");
                break;
            }
            if (ms < best) {
                best = ms;
                bT = T;
                bRB = RB;
                bcone = cone;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    ctx->cone_mode = cone0;
    if (st != TS_OK) return st;
    if (!bT) return fail(TS_EDEVICE, "no kernel configuration could be timed");
    apply_config(ctx, dtype, bT, bRB, 0);
    ctx->cone_mode = bcone;
    ctx->user_config[dtype] = true;
    if (ms_per_step) *ms_per_step = best;
    return TS_OK;
}

extern "C" ts_status ts_autotune(ts_ctx *ctx, ts_dtype dtype, int32_t order, void *scratch, int32_t use_cache,
                                 double *ms_per_step, void *stream)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (ctx->n < 1) {
        if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
        if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
        if (!scratch || !aligned(scratch, dtype)) return fail(TS_EINVAL, "scratch is NULL or misaligned");
        return autotune_batch(ctx, dtype, order, scratch, ms_per_step, static_cast<hipStream_t>(stream));
    }
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    if (!scratch || !aligned(scratch, dtype)) return fail(TS_EINVAL, "scratch is NULL or misaligned");
    if (ctx->n > (dtype == TS_C128 ? kMaxSpinsC128 : kMaxSpinsC64))
        return fail(TS_EINVAL, "too many spins for this dtype");
    ts_status st = ensure_device(ctx);
    if (st != TS_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const std::string arch = device_arch(), path = tune_cache_path();
    std::vector<TuneEntry> cache = read_tune_cache(path);
    if (use_cache) {
        for (const TuneEntry &e : cache)
            if (e.arch == arch && e.n == ctx->n && e.dtype == dtype && e.order == order &&
                valid_config(dtype, ctx->n, e.tile_bits, e.reg_bits, e.variant)) {
                apply_config(ctx, dtype, e.tile_bits, e.reg_bits, e.variant);
                ctx->tune_checked[dtype] = true;
                if (ms_per_step) *ms_per_step = e.ms;
                return TS_OK;
            }
    }
    // candidates: tile widths that keep runs of >= 128 bytes, both register widths, and the
    // LDS-staged kernel; each timed on one step (after one untimed step)
    const int hi = dtype == TS_C128 ? 13 : 14;
    struct Cand { int T, RB, v; };
    std::vector<Cand> cands;
    for (int T = 10; T <= hi; ++T) {
        for (int RB = 3; RB <= 4; ++RB)
            for (int v : {0, 2, 3, 4, 5})
                if (valid_config(dtype, ctx->n, T, RB, v)) cands.push_back({T, RB, v});
        if (T >= 11) cands.push_back({T, 4, 1});
    }
    hipEvent_t e0, e1;
    TS_HIP(hipEventCreate(&e0));
    TS_HIP(hipEventCreate(&e1));
    double best = 1e300;
    Cand bc{0, 0, 0};
    void *vec[1] = {scratch};
    for (const Cand &cd : cands) {
        apply_config(ctx, dtype, cd.T, cd.RB, cd.v);
        PlanEntry *pe;
        st = build_plan(ctx, dtype, cd.T, order, 0.01, 1, &pe);
        if (st == TS_OK) st = run_plan(ctx, pe, dtype, vec, 1, s);
        if (st != TS_OK) break;
        float ms = 0.f, m2 = 0.f;
        (void)hipEventRecord(e0, s);
        st = run_plan(ctx, pe, dtype, vec, 1, s);
        (void)hipEventRecord(e1, s);
        if (st != TS_OK) break;
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            st = fail(TS_EDEVICE, "timing failed");
            break;
        }
        (void)hipEventRecord(e0, s);
        st = run_plan(ctx, pe, dtype, vec, 1, s);
        (void)hipEventRecord(e1, s);
        if (st != TS_OK) break;
        if (hipEventSynchronize(e1) == hipSuccess && hipEventElapsedTime(&m2, e0, e1) == hipSuccess)
            ms = std::min(ms, m2);
        if (ms < best) {
            best = ms;
            bc = cd;
        }
        if (ctx->n <= cd.T) break;  // the state fits one tile: every candidate runs the same kernel
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != TS_OK) return st;
    if (!bc.T) return fail(TS_EDEVICE, "no kernel configuration could be timed");
    apply_config(ctx, dtype, bc.T, bc.RB, bc.v);
    ctx->tune_checked[dtype] = true;
    if (ms_per_step) *ms_per_step = best;
    std::vector<TuneEntry> out;
    for (const TuneEntry &e : cache)
        if (!(e.arch == arch && e.n == ctx->n && e.dtype == dtype && e.order == order)) out.push_back(e);
    TuneEntry ne;
    ne.arch = arch;
    ne.n = ctx->n;
    ne.dtype = dtype;
    ne.order = order;
    ne.tile_bits = bc.T;
    ne.reg_bits = bc.RB;
    ne.variant = bc.v;
    ne.ms = best;
    out.push_back(ne);
    (void)write_tune_cache(path, out);  // a cache that cannot be written only costs re-tuning
    return TS_OK;
}

extern "C" ts_status ts_create_batch(int32_t n_chains, const int32_t *n_spins, const ts_bond *bonds,
                                     const int32_t *bond_off, const double *fields, ts_ctx **out)
{
    if (!out) return fail(TS_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_chains < 1) return fail(TS_EINVAL, "n_chains must be >= 1");
    if (!n_spins || !bond_off) return fail(TS_EINVAL, "n_spins or bond_off is NULL");
    if (bond_off[0] != 0) return fail(TS_EINVAL, "bond_off[0] must be 0");
    for (int c = 0; c < n_chains; ++c)
        if (bond_off[c + 1] < bond_off[c]) return fail(TS_EINVAL, "bond_off must be non-decreasing");
    if (bond_off[n_chains] > 0 && !bonds) return fail(TS_EINVAL, "bonds is NULL");
    auto b = std::make_unique<ts_ctx>();
    int64_t foff = 0;
    for (int c = 0; c < n_chains; ++c) {
        ts_ctx *ch = nullptr;
        ts_status st = ts_create(n_spins[c], bonds ? bonds + bond_off[c] : nullptr,
                                 bond_off[c + 1] - bond_off[c], fields ? fields + 3 * foff : nullptr, &ch);
        if (st != TS_OK) return fail(st, "chain " + std::to_string(c) + ": " + g_err);
        foff += n_spins[c];
        ch->cone_mode = 0;   // a class's plans are formed together (build_batch_program)
        b->chains.emplace_back(ch);
    }
    b->n = 0;
    // batched classes keep the ping-pong sweeps unless asked (TSSPIN_CONE) or tuned otherwise:
    // with many chains per launch the GPU is full and the light-cone sweeps, bound by vector
    // instructions, measured slower on the 512-chain workload
    b->cone_mode = 0;
    if (const char *v = std::getenv("TSSPIN_CONE")) b->cone_mode = std::atoi(v);
    *out = b.release();
    return TS_OK;
}

extern "C" ts_status ts_evolve_batch(ts_ctx *ctx, void *psi_packed, const int64_t *psi_off, ts_dtype dtype,
                                     double dt, int64_t nsteps, int32_t order, const ts_observable *rec,
                                     int32_t n_rec, int32_t rec_every, double *rec_out, void *stream)
{
    if (!ctx || ctx->chains.empty()) return fail(TS_EINVAL, "ctx is not a batch context");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (!psi_packed || !psi_off) return fail(TS_EINVAL, "psi_packed or psi_off is NULL");
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    if (nsteps < 0) return fail(TS_EINVAL, "nsteps < 0");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    const int nch = (int)ctx->chains.size();
    for (int c = 0; c < nch; ++c) {
        if (psi_off[c] < 0) return fail(TS_EINVAL, "negative psi_off");
        if (ctx->chains[c]->n > (dtype == TS_C128 ? kMaxSpinsC128 : kMaxSpinsC64))
            return fail(TS_EINVAL, "too many spins for this dtype");
    }
    if (!aligned(psi_packed, dtype)) return fail(TS_EINVAL, "psi_packed is misaligned");
    std::vector<tsk::ObsDev> obs;
    int slots = 0;
    if (n_rec < 0 || n_rec > tsk::kMaxObs) return fail(TS_EINVAL, "n_rec must be 0..16");
    for (int k = 0; k < n_rec; ++k) {
        const ts_observable &o = rec[k];
        if (tsk::obs_complex(o.kind)) return fail(TS_EINVAL, "overlaps are not recorded in batches");
        if (o.kind == TS_OBS_ENERGY) return fail(TS_EINVAL, "the energy is not recorded in batches");
        for (int c = 0; c < nch; ++c) {
            std::vector<tsk::ObsDev> tmp;
            int s2 = 0;
            ts_status st = check_obs(ctx->chains[c].get(), &o, 1, 1, true, tmp, &s2);
            if (st != TS_OK) return fail(st, "chain " + std::to_string(c) + ": " + g_err);
        }
        obs.push_back(tsk::ObsDev{o.kind, o.i, o.j, 0, 0, slots});
        ++slots;
    }
    if (n_rec > 0 && (rec_every < 1 || !rec_out)) return fail(TS_EINVAL, "rec_every < 1 or rec_out is NULL");
    ts_status st = ensure_device(ctx);
    if (st != TS_OK) return st;
    for (auto &ch : ctx->chains) {
        st = ensure_device(ch.get());
        if (st != TS_OK) return st;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    // one program (and graph) per distinct call
    std::string key = std::to_string(dtype) + "|" + std::to_string(order) + "|" + std::to_string(nsteps) + "|" +
                      std::to_string(rec_every) + "|";
    uint64_t dtb;
    std::memcpy(&dtb, &dt, sizeof dtb);
    key += std::to_string(dtb) + "|" + std::to_string((uintptr_t)psi_packed) + "|" +
           std::to_string((uintptr_t)rec_out) + "|";
    for (const auto &o : obs) key += std::to_string(o.kind) + "," + std::to_string(o.i) + "," + std::to_string(o.j) + ";";
    key += "|cone" + std::to_string(ctx->cone_mode);
    for (int c = 0; c < nch; ++c) key += std::to_string(psi_off[c]) + ",";
    auto it = ctx->programs.find(key);
    BatchProgram *bp;
    if (it == ctx->programs.end()) {
        if (ctx->programs.size() >= (size_t)kMaxBatchPrograms) {
            // least recently used program out; its graph and buffers may still be in use
            // by queued work, so wait for the device first
            TS_HIP(hipDeviceSynchronize());
            ctx->programs.erase(ctx->program_order.front());
            ctx->program_order.erase(ctx->program_order.begin());
        }
        auto p = std::make_unique<BatchProgram>();
        st = build_batch_program(ctx, static_cast<char *>(psi_packed), psi_off, dtype, dt, nsteps, order, obs,
                                 slots, rec_every, rec_out, p.get());
        if (st != TS_OK) return st;
        TS_HIP(hipDeviceSynchronize());  // uploads done before capture
        if (!capture_batch_program(p.get())) ++ctx->capture_failures;
        bp = p.get();
        ctx->programs.emplace(key, std::move(p));
        ctx->program_order.push_back(key);
    } else {
        bp = it->second.get();
        auto o = std::find(ctx->program_order.begin(), ctx->program_order.end(), key);
        if (o != ctx->program_order.end()) std::rotate(o, o + 1, ctx->program_order.end());
    }
    if (bp->exec) {
        TS_HIP(hipGraphLaunch(bp->exec, s));
        ++ctx->graph_replays;
        return TS_OK;
    }
    // capture failed: the same launches, in order, on the caller's stream
    for (const auto &cl : bp->per_class)
        for (const BatchLaunch &L : cl) TS_HIP(run_launch(dtype, L, s));
    ++ctx->eager_runs;
    return TS_OK;
}

extern "C" ts_status ts_batch_stats(ts_ctx *ctx, int64_t *stats)
{
    if (!ctx || !stats) return fail(TS_EINVAL, "ctx or stats is NULL");
    stats[0] = ctx->graph_replays;
    stats[1] = ctx->eager_runs;
    stats[2] = ctx->capture_failures;
    stats[3] = (int64_t)ctx->programs.size();
    return TS_OK;
}

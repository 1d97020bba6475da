// tsspin.cpp -- C ABI of libtsspin: argument checks, the Hamiltonian tables, plan cache
// and kernel dispatch.  See include/tsspin.h for the contract of every entry point.
#include "../../include/tsspin.h"

#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstring>
#include <map>
#include <memory>
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
constexpr int kMaxSpinsC64 = 35;

int default_tile_bits(int dtype) { return dtype == TS_C128 ? 13 : 14; }
int min_run_bits(int dtype) { return dtype == TS_C128 ? 3 : 4; }  // 128-byte runs

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
};

struct PlanEntry {
    ts::Plan plan;
    DevBuf resident_ops;   // ResidentOp[] when plan.resident
    std::vector<tsk::DiagArgs> diag_args;  // one per chain diagonal
};

}  // namespace

struct ts_ctx {
    int n = 0;
    std::vector<int> bi, bj;                    // merged bonds, bi < bj
    std::vector<std::array<double, 3>> J;       // merged couplings
    std::vector<std::array<double, 3>> h;       // fields [n]
    bool zero_axis[3] = {false, false, false};
    int device = -1;
    int tile_bits[2] = {0, 0};                  // per dtype, 0 = default
    std::map<std::tuple<int, uint64_t, int>, std::unique_ptr<EnergyTable>> tables;
    std::map<std::tuple<int, int, int, uint64_t, int64_t>, std::unique_ptr<PlanEntry>> plans;
    DevBuf partials;       // reduction scratch
    DevBuf expect_out;     // ts_expect staging
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
    *out = t.get();
    c->tables.emplace(key, std::move(t));
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

ts_status build_plan(ts_ctx *c, int dtype, int T, int order, double dt, int64_t nsteps,
                     PlanEntry **out)
{
    uint64_t dtb;
    std::memcpy(&dtb, &dt, sizeof dtb);
    auto key = std::make_tuple(dtype, T, order, dtb, nsteps);
    auto it = c->plans.find(key);
    if (it != c->plans.end()) {
        *out = it->second.get();
        return TS_OK;
    }
    auto pe = std::make_unique<PlanEntry>();
    try {
        auto chain = ts::build_chain(order, dt, nsteps, c->zero_axis);
        pe->plan = ts::make_plan(chain, c->n, T, min_run_bits(dtype));
    } catch (const std::exception &e) {
        return fail(TS_EINVAL, std::string("plan: ") + e.what());
    }
    for (const auto &d : pe->plan.chain.diags) pe->diag_args.push_back(diag_args(d));
    *out = pe.get();
    c->plans.emplace(key, std::move(pe));
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

// Run one planned segment on every vector.
ts_status run_plan(ts_ctx *c, PlanEntry *pe, int dtype, void *const *psi, int n_psi,
                   hipStream_t stream)
{
    const ts::Plan &P = pe->plan;
    const int n = c->n;
    if (P.resident) {
        ts_status st = resident_ops(pe);
        if (st != TS_OK) return st;
        const int Tk = n < 8 ? 8 : n;
        // resident tables: no outside bits, geff = fields, jt = every coupling
        std::array<EnergyTable *, 3> tab{};
        for (int a = 0; a < 3; ++a) {
            if (c->zero_axis[a]) continue;
            st = get_table(c, Tk, (1ull << n) - 1, a, &tab[a]);
            if (st != TS_OK) return st;
        }
        tsk::ResidentArgs ra{};
        for (int v = 0; v < n_psi; ++v) ra.psi[v] = psi[v];
        ra.ops = static_cast<const tsk::ResidentOp *>(pe->resident_ops.p);
        ra.n_ops = (int)P.sweeps.size();
        ra.n = n;
        for (int a = 0; a < 3; ++a) {
            ra.wg[a] = tab[a] ? static_cast<const double *>(tab[a]->wg.p) : nullptr;
            ra.jt[a] = tab[a] ? static_cast<const double *>(tab[a]->jt.p) : nullptr;
        }
        TS_HIP(tsk::launch_resident(dtype, Tk, ra, n_psi, stream));
        return TS_OK;
    }
    const int T = P.tile_bits;
    for (const ts::Sweep &sw : P.sweeps) {
        tsk::SweepArgs a{};
        const uint64_t all = (1ull << n) - 1;
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
        const uint32_t nblocks = (uint32_t)(1ull << (n - T));
        for (int v = 0; v < n_psi; ++v) TS_HIP(tsk::launch_sweep(dtype, T, psi[v], a, nblocks, stream));
    }
    return TS_OK;
}

ts_status check_obs(const ts_ctx *c, const ts_observable *obs, int n_obs, int n_psi, bool in_evolve,
                    std::vector<tsk::ObsDev> &dev, int *slots)
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
        case TS_OBS_NORM: case TS_OBS_MZ: break;
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
            if (o.kind == TS_OBS_OVERLAP_SZ) {
                if (o.bra < 0 || o.bra >= n_psi) return fail(TS_EINVAL, "observable bra index out of range");
                d.bra = o.bra;
            }
        } else {
            d.ket = 0;
            if (o.kind == TS_OBS_OVERLAP_SZ) {
                if (!o.other) return fail(TS_EINVAL, "overlap observable needs `other`");
                d.bra = 1 + k;  // filled by the caller
            }
        }
        s += (o.kind == TS_OBS_OVERLAP_SZ) ? 2 : 1;
        dev.push_back(d);
    }
    *slots = s;
    return TS_OK;
}

constexpr int kRedBlocks = 1024;

ts_status reduce(ts_ctx *c, int dtype, const void *const *vecs, int nvec,
                 const std::vector<tsk::ObsDev> &obs, double *out, hipStream_t stream)
{
    tsk::ReduceArgs ra{};
    for (int v = 0; v < nvec; ++v) ra.psi[v] = vecs[v];
    for (size_t k = 0; k < obs.size(); ++k) ra.obs[k] = obs[k];
    ra.n_obs = (int)obs.size();
    ra.n = c->n;
    ts_status st = alloc(c->partials, (size_t)kRedBlocks * 2 * tsk::kMaxObs * sizeof(double));
    if (st != TS_OK) return st;
    const uint64_t dim = 1ull << c->n;
    uint64_t nb = dim / (256 * 4);
    if (nb < 1) nb = 1;
    if (nb > (uint64_t)kRedBlocks) nb = kRedBlocks;
    TS_HIP(tsk::launch_reduce(dtype, ra, static_cast<double *>(c->partials.p), (int)nb, out, stream));
    return TS_OK;
}

bool aligned(const void *p, int dtype) { return ((uintptr_t)p % (dtype == TS_C128 ? 16 : 8)) == 0; }

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
            c->bi.push_back(p);
            c->bj.push_back(q);
            c->J.push_back({b.jx, b.jy, b.jz});
        } else {
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
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int T = ctx->tile_bits[dtype] > 0 ? ctx->tile_bits[dtype] : default_tile_bits(dtype);
    const void *const *cpsi = const_cast<const void *const *>(psi);

    int64_t seg = n_rec > 0 ? rec_every : nsteps;
    int64_t nseg = (n_rec > 0 && seg > 0) ? nsteps / seg : (nsteps > 0 ? 1 : 0);
    int64_t rem = n_rec > 0 ? nsteps % seg : 0;
    if (n_rec > 0) {
        st = reduce(ctx, dtype, cpsi, n_psi, obs, rec_out, s);
        if (st != TS_OK) return st;
    }
    if (nseg > 0) {
        PlanEntry *pe;
        st = build_plan(ctx, dtype, T, order, dt, seg, &pe);
        if (st != TS_OK) return st;
        for (int64_t k = 0; k < nseg; ++k) {
            st = run_plan(ctx, pe, dtype, psi, n_psi, s);
            if (st != TS_OK) return st;
            if (n_rec > 0) {
                st = reduce(ctx, dtype, cpsi, n_psi, obs, rec_out + (size_t)(k + 1) * slots, s);
                if (st != TS_OK) return st;
            }
        }
    }
    if (rem > 0) {
        PlanEntry *pe;
        st = build_plan(ctx, dtype, T, order, dt, rem, &pe);
        if (st != TS_OK) return st;
        st = run_plan(ctx, pe, dtype, psi, n_psi, s);
        if (st != TS_OK) return st;
    }
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
        if (obs[k].kind == TS_OBS_OVERLAP_SZ) {
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

ts_status ts_plan_describe(ts_ctx *ctx, ts_dtype dtype, double dt, int64_t nsteps, int32_t order,
                           int32_t tile_bits, int64_t *out, int64_t cap, int64_t *n_sweeps)
{
    if (!ctx || !n_sweeps) return fail(TS_EINVAL, "ctx or n_sweeps is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    if (order != 1 && order != 2 && order != 4) return fail(TS_EINVAL, "order must be 1, 2 or 4");
    if (nsteps < 1) return fail(TS_EINVAL, "nsteps must be >= 1");
    if (!std::isfinite(dt)) return fail(TS_EINVAL, "dt is not finite");
    const int T = tile_bits > 0 ? tile_bits : default_tile_bits(dtype);
    if (T < 2 || T > 20) return fail(TS_EINVAL, "tile_bits out of range");
    ts::Plan P;
    try {
        auto chain = ts::build_chain(order, dt, nsteps, ctx->zero_axis);
        P = ts::make_plan(chain, ctx->n, T, min_run_bits(dtype));
    } catch (const std::exception &e) {
        return fail(TS_EINVAL, std::string("plan: ") + e.what());
    }
    *n_sweeps = (int64_t)P.sweeps.size();
    if (!out) return TS_OK;
    for (int64_t k = 0; k < *n_sweeps && k < cap; ++k) {
        const ts::Sweep &s = P.sweeps[k];
        int64_t *r = out + 12 * k;
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
    }
    return TS_OK;
}

}  // extern "C"

extern "C" ts_status ts_set_tile_bits(ts_ctx *ctx, ts_dtype dtype, int32_t tile_bits)
{
    if (!ctx) return fail(TS_EINVAL, "ctx is NULL");
    if (dtype != TS_C128 && dtype != TS_C64) return fail(TS_EINVAL, "unknown dtype");
    const int hi = dtype == TS_C128 ? 13 : 14;
    if (tile_bits != 0 && (tile_bits < 8 || tile_bits > hi))
        return fail(TS_EINVAL, "tile_bits must be 0 or 8..13 (c128) / 8..14 (c64)");
    ctx->tile_bits[dtype] = tile_bits;
    return TS_OK;
}

// plan.cpp -- schedule builder, layer folding and sweep planner (host only).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

namespace ts {

namespace {

const double kR = 0.70710678118654752440;  // 1/sqrt2
const cplx kI(0.0, 1.0);

// One-spin rotations of Sec. 2, Eq. Rotations, rewritten in the (down, up) index order
// used by the state vector (index 0 = bit clear = down):
//   R^x_{-pi/2} = (1/sqrt2)[[1, i], [i, 1]]    satisfies R^dagger S^y R = S^z
//   R^y_{pi/2}  = (1/sqrt2)[[1, 1], [-1, 1]]   satisfies R^dagger S^x R = S^z
// exp(-i t H_y) = X exp(-i t D_y) X^dagger with X = (x)R^x, and
// exp(-i t H_x) = Y exp(-i t D_x) Y^dagger with Y = (x)R^y.
M2 rot_x() { return {kR, kR * kI, kR * kI, kR}; }
M2 rot_y() { return {kR, kR, -kR, kR}; }

M2 dagger(const M2 &a) { return {std::conj(a[0]), std::conj(a[2]), std::conj(a[1]), std::conj(a[3])}; }

// b after a: the matrix of "apply a, then b".
M2 then(const M2 &a, const M2 &b)
{
    return {b[0] * a[0] + b[1] * a[2], b[0] * a[1] + b[1] * a[3],
            b[2] * a[0] + b[3] * a[2], b[2] * a[1] + b[3] * a[3]};
}

bool is_identity(const M2 &a)
{
    return std::abs(a[0] - 1.0) < 1e-12 && std::abs(a[1]) < 1e-12 && std::abs(a[2]) < 1e-12 &&
           std::abs(a[3] - 1.0) < 1e-12;
}

// c such that z = i^c, for |z| = 1 on an axis; -1 otherwise.
int quarter_code(cplx z)
{
    const cplx q[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};
    for (int c = 0; c < 4; ++c)
        if (std::abs(z - q[c]) < 1e-12) return c;
    return -1;
}

}  // namespace

bool step_substeps(int order, double dt, std::vector<std::pair<int, double>> &out)
{
    if (order == 1) {
        out.push_back({AX_Z, dt});
        out.push_back({AX_Y, dt});
        out.push_back({AX_X, dt});
        return true;
    }
    if (order == 2) {
        // U2(t) = U1^dagger(-t/2) U1(t/2): U1(t/2) acts first (z, y, x), then
        // U1^dagger(-t/2) = exp(-it/2 H_z) exp(-it/2 H_y) exp(-it/2 H_x) (x, y, z).
        const double h = 0.5 * dt;
        const int seq[6] = {AX_Z, AX_Y, AX_X, AX_X, AX_Y, AX_Z};
        for (int a : seq) out.push_back({a, h});
        return true;
    }
    if (order == 4) {
        const double a = 1.0 / (4.0 - std::cbrt(4.0));
        const double t[5] = {a * dt, a * dt, (1.0 - 4.0 * a) * dt, a * dt, a * dt};
        for (double ti : t) step_substeps(2, ti, out);
        return true;
    }
    return false;
}

std::vector<ChainOp> build_chain(int order, double dt, int64_t nsteps, const bool zero_axis[3],
                                 bool inverse)
{
    std::vector<std::pair<int, double>> sub;
    if (!step_substeps(order, dt, sub)) throw std::invalid_argument("order must be 1, 2 or 4");
    if (inverse) {
        std::reverse(sub.begin(), sub.end());
        for (auto &st : sub) st.second = -st.second;
    }
    std::vector<ChainOp> raw;
    const M2 X = rot_x(), Y = rot_y();
    for (int64_t s = 0; s < nsteps; ++s) {
        for (auto [axis, tau] : sub) {
            if (zero_axis[axis]) continue;
            ChainOp d;
            d.diag = true;
            d.axis = axis;
            d.tau = tau;
            if (axis == AX_Z) {
                raw.push_back(d);
                continue;
            }
            const M2 &R = (axis == AX_Y) ? X : Y;
            ChainOp l1, l2;
            l1.m = dagger(R);   // to the z frame
            l2.m = R;           // back
            raw.push_back(l1);
            raw.push_back(d);
            raw.push_back(l2);
        }
    }
    // Simplify until stable: multiply adjacent layers, drop identities, merge phases.
    for (bool changed = true; changed;) {
        changed = false;
        std::vector<ChainOp> out;
        for (const ChainOp &op : raw) {
            if (!out.empty() && !op.diag && !out.back().diag) {
                out.back().m = then(out.back().m, op.m);
                changed = true;
                if (is_identity(out.back().m)) out.pop_back();
                continue;
            }
            if (!out.empty() && op.diag && out.back().diag) {
                if (out.back().axis != op.axis)
                    throw std::runtime_error("internal: phases of two axes in one frame");
                out.back().tau += op.tau;
                changed = true;
                continue;
            }
            out.push_back(op);
        }
        raw.swap(out);
    }
    return raw;
}

FoldedChain fold_chain(const std::vector<ChainOp> &chain_in, int n)
{
    std::vector<ChainOp> chain = chain_in;
    // Normal form: begin and end with a phase step (an identity phase where needed).
    ChainOp id;
    id.diag = true;
    id.axis = AX_NONE;
    id.tau = 0.0;
    if (chain.empty() || !chain.front().diag) chain.insert(chain.begin(), id);
    if (!chain.back().diag) chain.push_back(id);

    FoldedChain fc;
    int carry_halves = 0;
    for (size_t k = 0; k < chain.size(); ++k) {
        const ChainOp &op = chain[k];
        if (!op.diag) continue;
        DiagStep d;
        d.axis = op.axis;
        d.tau = op.tau;
        int qt = 0, eighths = 0, halves = carry_halves;
        // layer before this phase: its left factor i^(cq*pop) and its scalar s^N
        if (k > 0 && !chain[k - 1].diag) {
            const M2 &m = chain[k - 1].m;
            cplx s = m[0];
            if (std::abs(std::abs(s) - kR) > 1e-12) throw std::runtime_error("layer scale");
            int cp = quarter_code(m[1] / s), cq = quarter_code(m[2] / s);
            if (cp < 0 || cq < 0 || std::abs(m[3] / s + (m[2] / s) * (m[1] / s)) > 1e-12)
                throw std::runtime_error("layer is not a butterfly");
            qt += cq;
            double ang = std::arg(s) / (M_PI / 4.0);
            long e8 = std::lround(ang);
            if (std::abs(ang - (double)e8) > 1e-9) throw std::runtime_error("layer phase");
            eighths += (int)(((e8 % 8) + 8) % 8) * (n % 8);
            halves += n;
            ++fc.n_layers;
        }
        // layer after this phase: its right factor i^(cp*pop)
        if (k + 1 < chain.size() && !chain[k + 1].diag) {
            const M2 &m = chain[k + 1].m;
            cplx s = m[0];
            int cp = quarter_code(m[1] / s);
            if (cp < 0) throw std::runtime_error("layer is not a butterfly");
            qt += cp;
        }
        d.qturn = qt & 3;
        d.eighths = eighths & 7;
        d.mag_exp = halves / 2;
        carry_halves = halves % 2;
        d.carry = carry_halves;
        fc.diags.push_back(d);
    }
    if (carry_halves) {
        fc.diags.back().mag_sqrt = 1;
        fc.diags.back().carry = 0;
    }
    return fc;
}

void plan_groups(int n, int T, int s_min, std::vector<uint64_t> &groups, std::vector<uint64_t> &tiles)
{
    groups.clear();
    tiles.clear();
    const uint64_t all = (n >= 64) ? ~0ull : ((1ull << n) - 1);
    if (n <= T) {
        groups.push_back(all);
        tiles.push_back(all);
        return;
    }
    groups.push_back((1ull << T) - 1);
    tiles.push_back((1ull << T) - 1);
    if (s_min > T - 1) s_min = T - 1;  // narrow tiles (tests): keep one rotated bit per group
    const int rest = n - T, per = T - s_min;
    const int ng = (rest + per - 1) / per;
    int lo = T;
    for (int g = 0; g < ng; ++g) {
        int sz = rest / ng + (g < rest % ng ? 1 : 0);
        uint64_t gm = ((1ull << sz) - 1) << lo;
        lo += sz;
        groups.push_back(gm);
        tiles.push_back(gm | ((1ull << (T - sz)) - 1));  // fill the tile with low bits
    }
}

Plan make_plan(const std::vector<ChainOp> &chain, int n, int T, int s_min, bool split_phases,
               bool balance)
{
    if (split_phases) {
        Plan p = make_plan(chain, n, T, s_min, false, balance);
        std::vector<Sweep> out;
        for (const Sweep &s : p.sweeps) {
            if (s.diag >= 0 && s.post_mask) {
                Sweep a = s, b = s;
                a.post_mask = 0;
                b.pre_mask = s.post_mask;
                b.post_mask = 0;
                b.diag = -1;
                out.push_back(a);
                out.push_back(b);
            } else {
                out.push_back(s);
            }
        }
        p.sweeps.swap(out);
        return p;
    }
    Plan p;
    p.n = n;
    p.tile_bits = (n < T) ? n : T;
    p.chain = fold_chain(chain, n);
    plan_groups(n, T, s_min, p.groups, p.tiles);
    const int g = (int)p.groups.size();
    const int m = p.chain.n_layers;
    p.resident = (g == 1);
    auto add = [&](int grp, bool pre, int diag, bool post) {
        Sweep s;
        s.group = grp;
        s.tile_mask = p.tiles[grp];
        s.pre_mask = pre ? p.groups[grp] : 0;
        s.post_mask = post ? p.groups[grp] : 0;
        s.diag = diag;
        p.sweeps.push_back(s);
    };
    if (g == 1) {
        // whole state in one tile: phase k then layer k+1, in one pass each
        for (int k = 0; k <= m; ++k) add(0, false, k, k < m);
        return p;
    }
    if (m == 0) {
        add(0, false, 0, false);
        return p;
    }
    for (int k = 1; k <= m; ++k) {
        const bool fwd = (k % 2) == 1;
        for (int idx = 0; idx < g; ++idx) {
            const int grp = fwd ? idx : g - 1 - idx;
            const bool first = idx == 0, last = idx == g - 1;
            if (first) {
                // layer k on the turning group was applied after phase k-1 (k > 1)
                if (k == 1) add(grp, false, 0, true);
                continue;
            }
            if (last) add(grp, true, k, k < m);
            else add(grp, true, -1, false);
        }
    }
    // Balance: the lowest index bits sit in every tile, and within one layer rotations of
    // different bits commute, so a layer-only sweep next to group 0's part of the same layer
    // can take those bits over (group 0's sweeps also carry a phase step and are the busiest).
    uint64_t everywhere = balance ? p.groups[0] : 0;
    for (uint64_t t : p.tiles) everywhere &= t;
    for (size_t i = 0; i < p.sweeps.size() && everywhere; ++i) {
        Sweep &s = p.sweeps[i];
        if (s.diag >= 0 || s.group == 0 || s.post_mask) continue;
        if (i > 0 && p.sweeps[i - 1].group == 0 && (p.sweeps[i - 1].post_mask & everywhere) == everywhere) {
            p.sweeps[i - 1].post_mask &= ~everywhere;   // same layer: after the phase of sweep i-1
            s.pre_mask |= everywhere;
        } else if (i + 1 < p.sweeps.size() && p.sweeps[i + 1].group == 0 &&
                   (p.sweeps[i + 1].pre_mask & everywhere) == everywhere) {
            p.sweeps[i + 1].pre_mask &= ~everywhere;    // same layer: before the phase of sweep i+1
            s.pre_mask |= everywhere;
        }
    }
    return p;
}

std::vector<BitRun> deposit_runs(uint64_t mask)
{
    std::vector<BitRun> runs;
    int src = 0;
    for (int b = 0; b < 64;) {
        if (!((mask >> b) & 1)) { ++b; continue; }
        int e = b;
        while (e < 64 && ((mask >> e) & 1)) ++e;
        runs.push_back({src, e - b, b});
        src += e - b;
        b = e;
    }
    return runs;
}

uint64_t deposit(uint64_t x, uint64_t mask)
{
    uint64_t r = 0;
    for (const BitRun &run : deposit_runs(mask))
        r |= ((x >> run.src) & ((1ull << run.len) - 1)) << run.dst;
    return r;
}

// ------------------------------------------------------------------ light-cone plan

bool make_cone_plan(const FoldedChain &fc, int n, int T, int s,
                    const std::vector<std::pair<int, int>> &bonds, int max_adv, size_t max_sweeps,
                    ConePlan &out, int max_phases)
{
    if (n <= T || n > 62 || s < 1 || s >= T) return false;
    const int m = fc.n_layers;
    if ((int)fc.diags.size() != m + 1) return false;
    // The butterflies gain sqrt2 per spin and layer; the folded scalars pay exactly that
    // back.  Here every phase step pays for the butterflies before it instead, and the
    // remaining unit-modulus part goes to the first phase step.
    long halves = 0;
    int e8 = 0;
    for (const DiagStep &d : fc.diags) {
        halves += 2L * d.mag_exp + d.mag_sqrt;
        e8 = (e8 + d.eighths) & 7;
    }
    if (halves != (long)n * m) return false;
    const int nb = (int)bonds.size();
    std::vector<std::vector<int>> inc(n);  // bonds of each spin
    for (int b = 0; b < nb; ++b) {
        const int i = bonds[b].first, j = bonds[b].second;
        if (i < 0 || j < 0 || i >= n || j >= n || i == j) return false;
        inc[i].push_back(b);
        inc[j].push_back(b);
    }
    std::vector<int> starts;
    for (int a = 0; a + T < n; a += T - s) starts.push_back(a);
    starts.push_back(n - T);
    const int nw = (int)starts.size();
    std::vector<int> order;
    for (int w = 0; w < nw; ++w) order.push_back(w);
    for (int w = nw - 2; w >= 1; --w) order.push_back(w);

    std::vector<int> level(n, 0), own_next(n, 0), bond_next(nb, 0), pos(n), start(n);
    for (int q = 0; q < n; ++q) pos[q] = q;
    int pend = 0;
    bool first_phase = true;
    auto all_done = [&]() {
        for (int q = 0; q < n; ++q)
            if (level[q] != m || own_next[q] != m + 1) return false;
        for (int b = 0; b < nb; ++b)
            if (bond_next[b] != m + 1) return false;
        return true;
    };
    auto low_spins = [&]() {  // spins at memory bits 0..s-1, in memory-bit order
        std::vector<int> lo(s, -1);
        for (int q = 0; q < n; ++q)
            if (pos[q] < s) lo[pos[q]] = q;
        return lo;
    };
    // Tile order, positions and the new memory bits of one sweep over the spins `win`.
    // next_low: the spins to put at memory bits 0..s-1 (in this order); home: every spin of
    // the window back to its own bit.
    auto emit = [&](const std::vector<int> &win, ConeSweep &sw, const std::vector<int> &next_low, bool home) {
        const std::vector<int> cur = low_spins();
        std::vector<char> used(n, 0), inwin(n, 0);
        for (int q : win) inwin[q] = 1;
        for (int q : cur) {
            if (q < 0 || !inwin[q]) return false;
        }
        std::vector<int> newpos(n);
        for (int q = 0; q < n; ++q) newpos[q] = pos[q];
        if (home) {
            for (int q : win) newpos[q] = q;
        } else {
            for (int i = 0; i < s; ++i) {  // swap next_low[i] and the spin at bit i
                const int a = next_low[i], b = cur[i];
                if (a == b) continue;
                if (!inwin[a]) return false;
                std::swap(newpos[a], newpos[b]);
            }
        }
        // tile order: the current low spins (lanes of the loads), then, when the low spins
        // change, fill up the register window and put the new low spins right after it
        // (lanes of the stores from window 0)
        std::vector<int> low_after(s, -1);
        for (int q : win) {
            if (newpos[q] < 0) return false;
            if (newpos[q] < s) low_after[newpos[q]] = q;
        }
        for (int q : low_after)
            if (q < 0) return false;
        const bool same_low = low_after == cur;
        sw.tile_q.clear();
        for (int q : cur) { sw.tile_q.push_back(q); used[q] = 1; }
        if (!same_low) {
            const int reg = std::max(s, 4);
            for (int q : win) {
                if ((int)sw.tile_q.size() >= reg) break;
                bool is_new = false;
                for (int x : low_after) is_new |= (x == q);
                if (!used[q] && !is_new) { sw.tile_q.push_back(q); used[q] = 1; }
            }
            if ((int)sw.tile_q.size() != reg) return false;
            for (int q : low_after) {
                if (used[q]) return false;
                sw.tile_q.push_back(q);
                used[q] = 1;
            }
        }
        for (int q : win)
            if (!used[q]) { sw.tile_q.push_back(q); used[q] = 1; }
        if ((int)sw.tile_q.size() != T) return false;
        sw.load_pos.resize(T);
        sw.store_pos.resize(T);
        uint64_t lset = 0, sset = 0;
        for (int i = 0; i < T; ++i) {
            sw.load_pos[i] = pos[sw.tile_q[i]];
            sw.store_pos[i] = newpos[sw.tile_q[i]];
            lset |= 1ull << sw.load_pos[i];
            sset |= 1ull << sw.store_pos[i];
        }
        if (lset != sset) return false;  // a store may only permute the tile's own bits
        sw.remap = sw.load_pos != sw.store_pos;
        for (int q : win) pos[q] = newpos[q];
        return true;
    };

    // The spins to hold the low memory bits after a sweep over [a, a + T) that is followed by
    // one over [an, an + T): the current ones if the next window holds them, else s spins
    // that both windows share (and that are not low now).
    auto choose_next = [&](int a, int an, std::vector<int> &next_low) {
        next_low.clear();
        const std::vector<int> cur = low_spins();
        bool keep = true;
        for (int q : cur) keep &= (q >= an && q < an + T);
        if (keep) {
            next_low = cur;
            return true;
        }
        for (int q = std::max(a, an); q < std::min(a, an) + T && (int)next_low.size() < s; ++q) {
            bool is_cur = false;
            for (int x : cur) is_cur |= (x == q);
            if (!is_cur) next_low.push_back(q);
        }
        return (int)next_low.size() == s;
    };
    int last_w = 0;
    out = ConePlan();
    out.n = n;
    out.T = T;
    out.s = s;
    out.chain = fc;
    out.bonds = bonds;
    size_t idle = 0;
    for (size_t it = 0; !all_done(); ++it) {
        if (out.sweeps.size() >= max_sweeps || idle > order.size()) return false;
        const int a = starts[order[it % order.size()]];
        const int an = starts[order[(it + 1) % order.size()]];
        std::vector<int> win;
        for (int q = a; q < a + T; ++q) win.push_back(q);
        auto inw = [&](int q) { return q >= a && q < a + T; };
        ConeSweep sw;
        for (int q : win) start[q] = level[q];
        int progress = 0;
        int lo = m;
        for (int q : win) lo = std::min(lo, level[q]);
        for (int k = lo; k <= m; ++k) {
            if (max_phases > 0 && (int)sw.phases.size() >= max_phases) break;
            ConePhase ph;
            ph.level = k;
            for (int q : win)
                if (level[q] == k && own_next[q] == k) {
                    ph.own |= 1ull << q;
                    own_next[q] = k + 1;
                }
            for (int b = 0; b < nb; ++b) {
                const int p = bonds[b].first, q = bonds[b].second;
                if (bond_next[b] == k && level[p] == k && level[q] == k && (inw(p) || inw(q))) {
                    ph.bonds.push_back(b);
                    bond_next[b] = k + 1;
                }
            }
            if (ph.own || !ph.bonds.empty()) {
                ph.half_scale = pend;
                pend = 0;
                if (first_phase) ph.eighths = e8;
                first_phase = false;
                ConeOp op;
                op.kind = 1;
                op.phase = (int)sw.phases.size();
                sw.ops.push_back(op);
                sw.phases.push_back(ph);
                ++progress;
            }
            if (k < m) {
                uint64_t A = 0;
                for (int q : win) {
                    if (level[q] != k || own_next[q] != k + 1) continue;
                    if (max_adv > 0 && level[q] - start[q] >= max_adv) continue;
                    bool ready = true;
                    for (int b : inc[q]) ready &= bond_next[b] == k + 1;
                    if (ready) A |= 1ull << q;
                }
                if (A) {
                    ConeOp op;
                    op.kind = 0;
                    op.spins = A;
                    sw.ops.push_back(op);
                    for (int q : win)
                        if ((A >> q) & 1) ++level[q];
                    pend += __builtin_popcountll(A);
                    ++progress;
                }
            }
            int hi = 0;
            for (int q : win) hi = std::max(hi, level[q]);
            if (k >= hi) break;
        }
        idle = progress ? 0 : idle + 1;
        const bool fin = all_done();
        std::vector<int> next_low;
        bool home = false;
        last_w = order[it % order.size()];
        if (fin) {
            bool can = true;
            for (int q = 0; q < n; ++q)
                if ((pos[q] != q || q < s) && !inw(q)) can = false;
            home = can;
            // otherwise the low spins move as for a step toward window 0; sweeps without
            // operations then walk back (below)
            if (!can && !choose_next(a, starts[std::max(last_w - 1, 0)], next_low)) return false;
        } else if (!choose_next(a, an, next_low)) {
            return false;
        }
        if (!emit(win, sw, next_low, home)) return false;
        out.sweeps.push_back(std::move(sw));
    }
    if (pend != 0) return false;
    // Back to every spin at its own bit: one sweep over the displaced spins when they fit a
    // tile, else sweeps without operations that retrace the windows toward window 0.
    for (int j = last_w - 1;; --j) {
        bool ident = true;
        for (int q = 0; q < n; ++q) ident &= pos[q] == q;
        if (ident) break;
        if (out.sweeps.size() >= max_sweeps) return false;
        std::vector<char> in(n, 0);
        int cnt = 0;
        for (int q = 0; q < n; ++q)
            if (pos[q] != q || pos[q] < s || q < s) { in[q] = 1; ++cnt; }
        std::vector<int> win;
        ConeSweep sw;
        if (cnt <= T) {
            for (int q = 0; q < n && cnt < T; ++q)
                if (!in[q]) { in[q] = 1; ++cnt; }
            for (int q = 0; q < n; ++q)
                if (in[q]) win.push_back(q);
            if (!emit(win, sw, {}, true)) return false;
            out.sweeps.push_back(std::move(sw));
            continue;
        }
        if (j < 0) return false;
        const int a = starts[j];
        for (int q = a; q < a + T; ++q) win.push_back(q);
        std::vector<int> next_low;
        if (!choose_next(a, starts[std::max(j - 1, 0)], next_low)) return false;
        if (!emit(win, sw, next_low, false)) return false;
        out.sweeps.push_back(std::move(sw));
    }
    for (int q = 0; q < n; ++q)
        if (pos[q] != q) return false;
    return true;
}

}  // namespace ts

// kernels.hpp -- argument blocks shared by the host engine and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace tsk {

constexpr int kMaxObs = 16;   // observables per reduction launch
constexpr int kMaxVec = 8;    // state vectors evolved in lockstep

// A run of consecutive bits: bits [src, src+len) of a dense index land on [dst, dst+len).
struct Run {
    int8_t src, len, dst, pad;
};

// One phase step: c_b *= kappa * i^(qturn*popcount(b)) * exp(-i tau D_axis(b)).
// axis < 0: no phase step; axis == 3: identity energy (only kappa and the quarter turns).
struct DiagArgs {
    int32_t axis;
    int32_t qturn;
    double tau;
    double kre, kim;
};

struct SweepArgs {
    Run tile_runs[4];   // tile index bits -> global bits
    Run out_runs[4];    // workgroup index bits -> global bits outside the tile
    int32_t n_tile_runs, n_out_runs;
    uint32_t pre_mask, post_mask;  // tile-index bits rotated before / after the phase
    DiagArgs d;
    const double *wg;   // [workgroups][T+1]: outside energy C, then geff per tile bit
    const double *jt;   // [T][T] couplings between tile bits (upper triangle used)
};

constexpr int kRegBits = 4;     // largest RB: amplitudes per thread = 2^RB in the register sweep
constexpr int kStagesPerWord = 7;
constexpr int kMaxStages = 2 * kStagesPerWord;

// 9-bit code of one stage: window start (bits 0-3), op (bit 4: 0 butterflies, 1 phase
// step), butterfly mask over the window bits (bits 5-8).  Stage s sits at bit 9*(s % 7) of
// st_code[s / 7]; the kernel decodes it with scalar shifts.
inline uint32_t stage_code(int win, int op, uint32_t mask)
{
    return (uint32_t)(win & 15) | ((uint32_t)(op & 1) << 4) | ((mask & 15u) << 5);
}

// One chain of a batched launch: its state, its workgroup phase factors and phase table
// for the sweep, and the base of its records (double[records][slots]).
struct ChainPtrs {
    void *psi;
    const double *wgf;
    const double *dtab;
    double *rec;
};

// Register-window sweep: stage s works in the layout whose register window starts at the
// coded tile bit and either applies butterflies on window bits or the phase step.
struct RegSweepArgs {
    Run tile_runs[4];
    Run out_runs[4];
    int32_t n_tile_runs, n_out_runs;
    uint64_t st_code[2];
    int32_t n_stages;
    int32_t load_win, store_win;  // layouts used for the global load and store
    int32_t diag_win;             // window of the phase step, -1 if none
    uint64_t n_tiles;             // tiles in the state; the pipelined grid may be smaller
    int32_t reverse;              // single state: workgroup w takes tile n_tiles - 1 - w
    // single state: the tile order is rotated by `rot` bits (then the low rot bits of the
    // workgroup index select the top bits of the tile index), 0 for none; see reg_sweep
    int32_t rot;
    void *psi2;                   // non-NULL: a second state in the same launch (grid doubled)
    uint64_t load_off[1 << kRegBits];   // global offset of register r in the load layout
    uint64_t store_off[1 << kRegBits];  // ... and in the store layout
    DiagArgs d;
    // Workgroup phase factors (re, im) [tiles][T+1]: exp(-i tau C), then exp(-i tau geff_k/2)
    // per tile bit (C, geff: outside energy and effective fields of the tile).  When the
    // phase step has no energy (identity axis, or no phase step) it points to a single
    // (1, 0) entry, which the kernels do not index.
    const double *wgf;
    const double *jt;
    // Host-built phase factors of this phase step (see diag_table in tsspin.cpp), as
    // (re, im) pairs: per thread pattern [1 + RB] then the window table [2^RB].
    const double *dtab;
    // Batched launch: chains[c] replaces psi, wgf and dtab for workgroups
    // c * tiles_per_chain .. (c + 1) * tiles_per_chain - 1.  NULL for a single state.
    const ChainPtrs *chains;
    uint64_t tiles_per_chain;
    // Energy-table variant: the phase step's energies D_axis(b) for every basis index b
    // (double for complex128, float for complex64; NULL when the step has no energy) and the
    // global offset of register r in the phase step's layout.
    const void *etab;
    uint64_t diag_off[1 << kRegBits];
};

// Light-cone sweep: one pass whose stage program applies butterflies and phase steps of
// several layers to the spins of one window, with arbitrary tile-bit -> memory-bit maps for
// the load and the store (the store may permute the tile's bits).  The arguments live in
// device memory (one block per sweep of a plan).
constexpr int kConeRuns = 16;
constexpr int kConeStages = 192;
constexpr int kConePhases = 24;
constexpr int kConeRowBits = 12;

// Stage code: window start (bits 0-3; a change of window is a transpose first), butterfly
// mask over the window bits (bits 5-8, may be 0), a phase step after the butterflies
// (bit 4), its index (bits 9-14) and the window bits v whose thread-table entry 1 + v the
// step reads (bits 15-18, cone_th_need).  32-bit words so that the kernel reads them with
// scalar loads.
inline uint32_t cone_code(int win, int has_phase, uint32_t mask, int phase)
{
    return (uint32_t)((win & 15) | ((has_phase & 1) << 4) | ((mask & 15u) << 5) | ((phase & 63) << 9));
}
// Thread-table entries 1 + v that a phase step with walk mask cmask reads: the specialised
// masks (0, the lowest or the highest window bit, or both) read their own bits, the general
// walk reads all four.
inline uint32_t cone_th_need(uint32_t cmask)
{
    return (cmask == 0 || cmask == 1 || cmask == 8 || cmask == 9) ? cmask : 15u;
}

struct ConePhaseArgs {
    double kre, kim;           // scalar of the step
    // Rows [2^n_row_bits][T+1] of (re, im), with geff_k the field that the step's bonds to
    // spins outside the tile put on tile bit k (the outside bits select the row; 0 for tile
    // bits without such bonds) and w the step's register window: entry 1+k is
    // exp(-i tau geff_k / 2) for k outside the window and exp(-i tau geff_k) for k in it,
    // entry 0 is exp(+i tau (sum of geff over the window) / 2) (every window bit down).
    const double *wgf;
    // (re, im) pairs: per thread pattern [1 + RB], then the window table [2^RB]: [0] the terms
    // among thread bits (fields, quarter turns, bonds) times exp(+i tau (sum of h_v) / 2),
    // [1+v] exp(-i tau h_v) with h_v the field of the thread bits' bonds on window bit v,
    // then per register the terms among window bits.  (The factors for every window bit
    // down, and the squares that flip one bit up, are the kernel's walk over the window.)
    const double *dtab;
    int8_t row_bit[kConeRowBits];  // workgroup-index bit of row bit i
    int32_t n_row_bits;
    uint32_t xmask;            // tile bits with a row-dependent field
    // Window bits v (of the step's register window) whose factor depends on the thread or
    // the workgroup: a bond of the step joins tile bit w + v to a tile bit outside the
    // window, or xmask has bit w + v.  For every other window bit the walk factor is
    // exactly 1 + 0i and the kernel skips it.
    uint32_t cmask;
};

struct ConeArgs {
    Run load_runs[kConeRuns];   // tile index bits -> memory bits when loading
    Run store_runs[kConeRuns];  // ... when storing
    Run out_runs[kConeRuns];    // workgroup index bits -> memory bits outside the tile
    int32_t n_load_runs, n_store_runs, n_out_runs;
    int32_t load_win, store_win;
    int32_t n_stages, n_phases;
    uint64_t load_off[1 << kRegBits];
    uint64_t store_off[1 << kRegBits];
    uint32_t st[kConeStages];
    ConePhaseArgs ph[kConePhases];
};

struct ResidentOp {
    DiagArgs d;
    int32_t post;       // 1: butterflies on every bit after the phase step
    int32_t rec;        // >= 0: record the observables as record `rec` after this op
    // non-NULL: the phase step's factor of every amplitude (2^n, from
    // launch_resident_factors), applied instead of forming it
    const double2 *fac;
};

struct ObsDev {
    int32_t kind, i, j, ket, bra, slot;
};

// Observables folded into the last light-cone sweep of a vector's recorded segment.  They
// need no amplitude but the one at b itself (and, for overlaps, the bra's amplitude at b):
// norm, S^z_i, S^z_i S^z_j, M^z, <bra|S^z_i|ket>, <bra|ket>.  The sweep stores its tile in
// the segment's final layout (every spin at its own bit), so each stored amplitude's address
// is its basis index b.  Workgroup w writes its FP64 sums of observable o to
// partials[w * 2 * kMaxObs + 2 * obs[o].slot + (0: real part, 1: imaginary part)] (here
// `slot` is the observable's column among all that the segment's sweeps fold in).
constexpr int kConeRecMax = 4;  // observables one vector's last sweep accumulates
struct ConeRec {
    ObsDev obs[kConeRecMax];
    const void *bra[kConeRecMax];   // overlaps: the bra vector (final), else unused
    int32_t n_obs;
    int32_t n;
    double *partials;
};

// One chain of a batched resident launch (one workgroup each).
struct ResidentChain {
    void *psi;
    const double *wg[3];
    const double *jt[3];
    double *rec;          // double[records][slots]
};

struct ResidentArgs {
    void *psi[kMaxVec];
    const ResidentOp *ops;
    int32_t n_ops;
    int32_t n;            // spins (<= T)
    const double *wg[3];  // per axis [T+1]: 0, then the field on each bit (NULL: axis unused)
    const double *jt[3];  // per axis [T][T]
    const ResidentChain *chains;  // batched: per-workgroup state, tables and records
    ObsDev obs[kMaxObs];          // observables of the record ops (real kinds)
    int32_t n_obs, slots;
    // One vector only: run the op list n_rep times (0 counts as 1) and, when rec_rows is
    // set, record the observables into rec_rows[r * slots ...] after repetition r.
    int32_t n_rep;
    double *rec_rows;
};

// Batched FP64 observables of many chains of one size (real kinds only).
struct BatchReduceArgs {
    const ChainPtrs *chains;
    ObsDev obs[kMaxObs];
    int32_t n_obs, n, rec, slots;
};

// One merged bond of the Hamiltonian for the energy observable (Sec. 2, Eq. 1).
struct HamBond {
    int32_t i, j;
    double jx, jy, jz;
};

// Observable kinds of ObsDev: the public ts_obs_kind values (0-8), and two that only the
// adjoint uses for the explicit terms of the energy gradient.
constexpr int kObsOverlapSz = 7;  // <bra|S^z_i|ket>, complex
constexpr int kObsOverlap = 8;    // <bra|ket>, complex
constexpr int kObsSxSx = 9;       // <S^x_i S^x_j>
constexpr int kObsSySy = 10;      // <S^y_i S^y_j>
__host__ __device__ constexpr bool obs_complex(int kind) { return kind == kObsOverlapSz || kind == kObsOverlap; }

struct ReduceArgs {
    const void *psi[kMaxVec];
    ObsDev obs[kMaxObs];
    int32_t n_obs;
    int32_t n;
    // the Hamiltonian, for the energy observable: fields [n][3] (x, y, z) and merged bonds
    const double *ham_h;
    const HamBond *ham_b;
    int32_t ham_nb;
};

// Adjoint: parameters of one axis whose gradient a reduction accumulates; pj < 0 marks a
// field on spin pi, otherwise a coupling of spins pi and pj.  Workgroup b adds
// coef * (its partial sum) to slots[b * stride + off + p]; the slots persist across the
// phase steps of a reverse pass and one final kernel sums them over workgroups.
constexpr int kGradChunk = 32;
struct GradArgs {
    int16_t pi[kGradChunk], pj[kGradChunk];
    int32_t np;         // parameters in this chunk
    int32_t n;          // spins
    double coef;        // 2 tau (forward sign) / (scale of the stored frame states)^2
    double *slots;      // [workgroups][stride]
    int32_t stride, off;
};

hipError_t launch_apply_obs(int dtype, const void *psi, void *out, int kind, int i, int j, int n,
                            hipStream_t s);
// out = H psi (H of Sec. 2, Eq. 1, from the fields [n][3] and merged bonds); out != psi.
hipError_t launch_apply_ham(int dtype, const void *psi, void *out, int n, const double *ham_h,
                            const HamBond *ham_b, int nb, hipStream_t s);
hipError_t launch_batch_reduce(int dtype, const BatchReduceArgs &a, int nchains, double *partials,
                               int nbpc, hipStream_t s);
// complex128 variant with half the LDS per workgroup (three workgroups per CU at T = 12).
hipError_t launch_sweep_half(int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s);
// Pipelined variant: a grid of resident workgroups, each prefetching its next tile.
hipError_t launch_sweep_pipe(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s);
hipError_t launch_sweep_reg_batch(int dtype, int T, int RB, const RegSweepArgs &a, uint32_t nchains,
                                  hipStream_t s);
hipError_t launch_grad_reduce(int dtype, const void *psi, const void *lam, const GradArgs &a,
                              int nblocks, hipStream_t s);

// Every parameter of one axis in one pass (n >= 10): workgroup w (one wave) owns amplitudes
// [w * 1024, (w + 1) * 1024) and adds coef * sum_b f_p(b) Im(conj(lam_b) psi_b) to
// slots[w * stride + off + col[p]] for p < np.  Lane t holds the amplitudes w * 1024 +
// e * 64 + t, e < 16 (index bits 6-9 vary along e).  The parameters come grouped by the set
// of their spins among bits 6-9 (group m: those spins are 6 + the bits of m;
// group_start[0..16] delimit the groups), with pi, pj their spins (pj < 0: a field).
struct GradWalshArgs {
    const int16_t *pi, *pj, *col;
    int32_t group_start[17];
    int32_t np, n;
    double coef;
    double *slots;
    int32_t stride, off;
};
// The adjoint's reverse sweep on psi and lambda together (one workgroup holds the same
// tile of both), with the gradient sums of the sweep's phase step taken in registers right
// after the step: coef * sum_b f_p(b) Im(conj(lam_b) psi_b) is added to
// slots[workgroup * stride + off + col[p]] for every parameter p < np of the step's axis.
// tile_bit[q] is the tile bit that holds spin q in this sweep, or -1 if q is outside the
// tile (its bit is then fixed for the workgroup).
struct PairGradArgs {
    const int16_t *pi, *pj, *col;
    int32_t np;
    double coef;
    double *slots;
    int32_t stride, off;
    int8_t tile_bit[64];
};
// Register-window sweep whose phase step reads the energies from a table in HBM (one per
// axis, 2^N entries) instead of forming them from the workgroup, thread and window tables.
hipError_t launch_sweep_etab(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s);
// out[b] = D_axis(b) = sum_i h[3 i + axis] s_i(b) + sum_bonds J_axis s_i(b) s_j(b), s = bit - 1/2,
// for b < 2^n; out is double (dtype 0) or float (dtype 1).
hipError_t launch_energy_table(int dtype, void *out, int n, const double *h, const HamBond *bonds, int n_bonds,
                               int axis, hipStream_t s);
hipError_t launch_sweep_pair(int dtype, int T, int RB, void *psi, void *lam, const RegSweepArgs &a,
                             const PairGradArgs &g, hipStream_t s);

constexpr int kGradWalshElems = 16;    // amplitudes per lane, 64 apart
constexpr int kGradWalshBlock = 64;    // one wave per workgroup
constexpr int kGradWalshLow = 6;       // the lowest index bit that varies along a lane's amplitudes
hipError_t launch_grad_walsh(int dtype, const void *psi, const void *lam, const GradWalshArgs &a,
                             hipStream_t s);
// out[c] = sum over workgroups b (fixed order) of slots[b * ncols + c], c < ncols.
hipError_t launch_grad_finalize(const double *slots, int nblocks, int ncols, double *out, hipStream_t s);

// Adjoint light-cone sweep: psi and lambda run through one stage program in the same
// workgroup (the inverse chain of the forward run), and after each phase step the gradient
// sums of the step's own terms are taken in registers.  The state in the sweep carries the
// butterflies' gain 2^(e/2) not yet paid back by the steps' scalars, the same for every
// amplitude and both vectors, so a step's sums are scaled by coef = -2 tau / 2^e.
constexpr int kConeGradSlots = 128;   // parameters (axis and field or bond) one sweep touches
constexpr int kConeGradTerms = 64;    // terms of one phase step
// The kernel reads a phase step's terms and offsets lane by lane (one vector load each) and
// takes them from there with readlane, so the term loop waits on no memory.
struct ConeGradArgs {
    double coef[kConePhases];          // per phase step; 0 for steps without an energy axis
    // terms of step p whose spins inside the register window form the mask m are
    // term[p][start[p][m]] .. term[p][start[p][m + 1] - 1]
    int32_t start[kConePhases][32];
    // one term: word 0 = accumulator (bits 0-7), the number of the term's spins outside the
    // register window (bits 8-9) and the mask of those that are tile bits (bits 12-31, a
    // thread's index bits); word 1 = the mask of those that are bits of the workgroup's tile
    // index.  The term's factor is then 2^-count * (-1)^(number of masked bits that are 0).
    uint32_t term[kConePhases][2][kConeGradTerms];
    int32_t n_slots;
    int32_t col[kConeGradSlots];       // column of each accumulator in the gradient row
};
// One adjoint light-cone sweep of psi and lam; g (device) the sweep's terms; workgroup w adds
// its sums to slots[w * stride + col[s]].
hipError_t launch_cone_pair(int dtype, int T, int RB, void *psi, void *lam, const ConeArgs *a, int n_phases,
                            const ConeGradArgs *g, int n_slots, double *slots, int stride, uint64_t n_tiles,
                            int reverse, hipStream_t s);

// One light-cone sweep of n_tiles workgroups; `a` points to device memory and n_phases is its
// n_phases (checked against the limit).  The phase tables that `a` names are read-only while
// the sweep runs (the kernel reads them through the scalar data cache).
hipError_t launch_cone(int dtype, int T, int RB, void *psi, const ConeArgs *a, int n_phases,
                       uint64_t n_tiles, int reverse, hipStream_t s);
// The same sweep with the observables of `rec` accumulated from the stored tile (one row of
// rec.partials per workgroup).
hipError_t launch_cone_rec(int dtype, int T, int RB, void *psi, const ConeArgs *a, int n_phases,
                           uint64_t n_tiles, int reverse, const ConeRec &rec, hipStream_t s);
// Sum the partial rows of nblocks workgroups into out[slot] (fixed order, compensated), for
// the observables (and slots) of `a`.  Beyond 1024 rows a first pass sums groups of 1024
// rows into `tmp` (ceil(nblocks / 1024) rows of 2 * kMaxObs doubles).
hipError_t launch_finalize(const double *partials, int nblocks, const ReduceArgs &a, double *out,
                           double *tmp, hipStream_t s);
// The same sweep for many chains of one size at once: chain c's state starts at element
// off[c] of `packed` and its arguments for this sweep are args[c] (device memory);
// tiles_per_chain workgroups per chain.
hipError_t launch_cone_batch(int dtype, int T, int RB, void *packed, const int64_t *off,
                             const ConeArgs *args, uint32_t nchains, uint64_t tiles_per_chain, int reverse,
                             hipStream_t s);
hipError_t launch_sweep(int dtype, int T, void *psi, const SweepArgs &a, uint32_t nblocks,
                        hipStream_t s);
hipError_t launch_sweep_reg(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s);
hipError_t launch_resident(int dtype, int T, const ResidentArgs &a, int nvec, hipStream_t s);
// The phase factors of a's ops (one vector's tables; every op with a phase step): op k's
// factor of amplitude t to out[k * 2^n + t].  T <= 13.
hipError_t launch_resident_factors(int T, const ResidentArgs &a, double2 *out, hipStream_t s);
hipError_t launch_reduce(int dtype, const ReduceArgs &a, double *partials, int nblocks,
                         double *out, hipStream_t s);

// Fixed reduction scratch of the allocation-free entry point (ts_expect_noalloc): the
// per-workgroup partials of at most kScratchBlocks workgroups, 2 * kMaxObs doubles each
// (256 KiB on every GPU the library runs on, held until the process ends).
constexpr int kScratchBlocks = 1024;
constexpr size_t kScratchDoubles = (size_t)kScratchBlocks * 2 * kMaxObs;
// Device address of the current GPU's copy of that array, looked up once per device (with
// the device current) and kept.
hipError_t scratch_address(double **out);

}  // namespace tsk

// plan.hpp -- host-side schedule builder and sweep planner of libtsspin.
//
// A run of Trotter steps (Sec. 2: U1, U2, U4) is first written as a chain of partial
// evolutions, each exp(-i tau H_a) as [rotate every spin to the a frame] [phase
// exp(-i tau D_a)] [rotate back] (Sec. 2, Eqs. Single Spin Rotation and
// Two-Spin-Operators; Sec. 3 "Forward Rotation -> Phases in Z -> Backward Rotation").
// The chain is then simplified: back-to-back rotations are multiplied into one layer,
// layers that cancel are dropped and phases of one axis that become adjacent are merged.
//
// Every remaining layer is the same 2x2 matrix M on every spin, and each one that occurs
// factors as M = s * diag(1, q) * [[1, 1], [1, -1]] * diag(1, p) with p, q in {1, i, -1, -i}
// and |s| = 1/sqrt2.  Over all spins that is s^N * i^(cq*popcount) * WHT * i^(cp*popcount):
// an unnormalised Walsh-Hadamard transform framed by diagonal quarter-turn phases.  The
// diagonal factors and the scalars commute with the neighbouring phase step and are folded
// into it, so a rotation layer costs only the add/subtract butterfly (u+v, u-v) per pair.
//
// The planner then cuts every layer into bit groups that fit one workgroup tile (the
// closed sets of Sec. 3.3) and orders them so that consecutive layers turn around on the
// same group ("ping-pong"): a sweep over the state applies [layer k on group G] [phase k]
// [layer k+1 on group G].  Low bits always stay inside a tile so every workgroup moves
// contiguous runs (the coalescing rule of Sec. 3.4).
#pragma once

#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace ts {

using cplx = std::complex<double>;
using M2 = std::array<cplx, 4>;  // row-major 2x2

enum { AX_X = 0, AX_Y = 1, AX_Z = 2, AX_NONE = 3 };

// One link of the chain, in the order the operations act on the state.
struct ChainOp {
    bool diag = false;
    int axis = AX_NONE;  // diagonal: which energy D_a
    double tau = 0.0;    // diagonal: time of exp(-i tau D_a)
    M2 m{};              // layer: the per-spin 2x2 matrix
};

// Sub-steps (axis, tau) of one Trotter step of order 1, 2 or 4, in application order.
// Returns false for another order.
bool step_substeps(int order, double dt, std::vector<std::pair<int, double>> &out);

// Build and simplify the chain of nsteps steps.  zero_axis[a] drops the partial evolutions
// of an axis whose part of H vanishes (they are the identity).  inverse = true builds the
// exact inverse of the same run: the sub-steps of each step in reverse order with -tau
// (for the palindromic orders 2 and 4 that equals the run with -dt; for order 1 it does not).
std::vector<ChainOp> build_chain(int order, double dt, int64_t nsteps, const bool zero_axis[3],
                                 bool inverse = false);

// Parameters of one phase step after folding the layer factors in: the diagonal
// multiplies c_b by  kappa * i^(qturn*popcount(b)) * exp(-i tau D_axis(b))  with
// kappa = 2^-mag_exp * (1/sqrt2)^mag_sqrt * exp(i pi eighths/4).
struct DiagStep {
    int axis = AX_NONE;
    double tau = 0.0;
    int qturn = 0;
    int mag_exp = 0;
    int mag_sqrt = 0;
    int eighths = 0;
    // After this phase step the state equals the true state (up to diagonal unit-modulus
    // factors) times 2^(carry/2): the butterflies' gain not yet paid back.
    int carry = 0;
};

// Chain in normal form: diag[0], layer, diag[1], layer, ..., layer, diag[m]; m >= 0 layers.
struct FoldedChain {
    std::vector<DiagStep> diags;  // m + 1 entries
    int n_layers = 0;
};

// Fold the layer factors of a chain into its diagonals for an N-spin register.  Throws
// std::runtime_error if a layer is not of the butterfly form above.
FoldedChain fold_chain(const std::vector<ChainOp> &chain, int n);

// One pass over the state vector.
struct Sweep {
    int group = 0;
    uint64_t tile_mask = 0;   // global bits resident in a tile
    uint64_t pre_mask = 0;    // bits given the butterfly before the diagonal
    uint64_t post_mask = 0;   // bits given the butterfly after the diagonal
    int diag = -1;            // index into FoldedChain::diags, or -1
};

struct Plan {
    int n = 0;
    int tile_bits = 0;                // T
    std::vector<uint64_t> groups;     // rotated bits of each group
    std::vector<uint64_t> tiles;      // tile mask of each group
    FoldedChain chain;
    std::vector<Sweep> sweeps;
    bool resident = false;            // n <= T: one workgroup holds the whole state
};

// Group layout for n spins, tile of T bits, at least s_min low bits in every tile.
void plan_groups(int n, int T, int s_min, std::vector<uint64_t> &groups,
                 std::vector<uint64_t> &tiles);

// Full plan of one chain.  With split_phases every phase step ends its sweep (the layer
// after it gets a sweep of its own), so the state in memory between those two sweeps is in
// the frame of that phase step; the adjoint reads it there.  With balance the rotations of
// the low bits shared by every tile move from the low group's sweeps (which also carry a
// phase step) to the neighbouring sweep of the same layer; the result is the same.
Plan make_plan(const std::vector<ChainOp> &chain, int n, int T, int s_min, bool split_phases = false,
               bool balance = true);

// Runs of consecutive bits of a mask: (source bit, length, destination bit) triples that
// scatter the bits of a dense index into the positions of the mask (a bit deposit).
struct BitRun {
    int src, len, dst;
};
std::vector<BitRun> deposit_runs(uint64_t mask);
uint64_t deposit(uint64_t x, uint64_t mask);

}  // namespace ts

namespace ts {

// ------------------------------------------------------------------ light-cone plan
//
// Every layer is a product of one-spin butterflies and every phase step a product of
// one-spin terms (field, quarter turn) and two-spin terms (one per bond), all diagonal.
// Operations on different spins commute, so a spin may run several layers ahead of a
// spin it is not coupled to: spin q may take layer k+1 once every level-k term that
// touches it has been applied, and a level-k bond term needs both of its spins at level
// k.  For a Hamiltonian whose bonds join spins that are close in index order (chains),
// a sweep over a window of T spins can then advance the middle of the window by many
// layers (a light cone bounded by the spins just outside it), instead of one layer part
// per sweep.  Bond terms to a spin outside the window use its fixed bit: an effective
// field per workgroup.
//
// Windows are intervals of spins.  Each tile must contain the s lowest memory bits
// (contiguous runs), so the spins stored there are remapped as the windows move: a sweep
// may store its tile with a permutation of the tile's own bits, which moves s spins that
// the next window shares into the low memory bits.  A plan starts and ends with every
// spin at its own bit.

struct ConePhase {
    int level = 0;              // index into FoldedChain::diags
    uint64_t own = 0;           // spins whose field and quarter-turn terms of the level apply
    std::vector<int> bonds;     // bonds (indices) whose term of the level applies
    int half_scale = 0;         // the step's scalar has modulus (1/sqrt2)^half_scale
    int eighths = 0;            // ... and phase exp(i pi eighths / 4)
};

struct ConeOp {
    int kind = 0;               // 0: butterflies on the spins of `spins`; 1: phase step `phase`
    uint64_t spins = 0;
    int phase = -1;
};

struct ConeSweep {
    std::vector<int> tile_q;      // spin held by tile bit i, i < T
    std::vector<int> load_pos;    // memory bit of tile bit i when the tile is loaded
    std::vector<int> store_pos;   // ... and when it is stored
    std::vector<ConeOp> ops;
    std::vector<ConePhase> phases;
    bool remap = false;           // store_pos differs from load_pos
};

struct ConePlan {
    int n = 0, T = 0, s = 0;
    FoldedChain chain;
    std::vector<std::pair<int, int>> bonds;
    std::vector<ConeSweep> sweeps;
};

// Light-cone plan of a folded chain for n spins, tiles of T bits of which the s lowest
// memory bits are in every tile, bonds (i, j) as listed (duplicates allowed).  max_adv
// bounds the layers one spin takes in one sweep and max_phases the phase steps of one sweep
// (<= 0: no bound).  Returns false (and
// leaves `out` unspecified) when the windows cannot cover the spins under these rules:
// n <= T, s >= T, or a plan longer than max_sweeps.
bool make_cone_plan(const FoldedChain &fc, int n, int T, int s,
                    const std::vector<std::pair<int, int>> &bonds, int max_adv, size_t max_sweeps,
                    ConePlan &out, int max_phases = 0);

}  // namespace ts

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

struct ResidentOp {
    DiagArgs d;
    int32_t post;       // 1: butterflies on every bit after the phase step
    int32_t pad;
};

struct ResidentArgs {
    void *psi[kMaxVec];
    const ResidentOp *ops;
    int32_t n_ops;
    int32_t n;            // spins (<= T)
    const double *wg[3];  // per axis [T+1]: 0, then the field on each bit (NULL: axis unused)
    const double *jt[3];  // per axis [T][T]
};

struct ObsDev {
    int32_t kind, i, j, ket, bra, slot;
};

struct ReduceArgs {
    const void *psi[kMaxVec];
    ObsDev obs[kMaxObs];
    int32_t n_obs;
    int32_t n;
};

hipError_t launch_sweep(int dtype, int T, void *psi, const SweepArgs &a, uint32_t nblocks,
                        hipStream_t s);
hipError_t launch_resident(int dtype, int T, const ResidentArgs &a, int nvec, hipStream_t s);
hipError_t launch_reduce(int dtype, const ReduceArgs &a, double *partials, int nblocks,
                         double *out, hipStream_t s);

}  // namespace tsk

/*
 * tsspin.h -- C ABI of libtsspin: fourth-order fractal-Suzuki Trotter evolution of a full
 * 2^N spin-1/2 state vector under the XYZ decomposition, on one AMD MI355X (gfx950) GPU.
 *
 * Paper: A. D. Dente, C. S. Bederian, P. R. Zangara, H. M. Pastawski, "GPU accelerated
 * Trotter-Suzuki solver for quantum spin dynamics", arXiv:1305.0036.
 *
 * Conventions used by every call (Sec. 2, Eqs. 1-2; Sec. 3.2 footnote; Sec. 3.3 example):
 *   - The Hamiltonian is H = sum_j sum_a h^a_j S^a_j + sum_bonds sum_a J^a_ij S^a_i S^a_j,
 *     a in {x, y, z}, S = sigma/2, hbar = 1.  Each bond is an unordered pair i != j counted
 *     once; bonds listed twice are summed (Eq. 1 is a sum).
 *   - The state holds the 2^N Ising-basis coefficients c_b.  Spin j is bit j of b (bit 0 =
 *     spin counted first from the right).  A set bit is spin up, s_j = +1/2.
 *   - H is split by axis into H_x, H_y, H_z (field and coupling terms of one axis together).
 *     U1(t) = exp(-itH_x) exp(-itH_y) exp(-itH_z) (Eq. U1: the z part acts first),
 *     U2(t) = U1^dagger(-t/2) U1(t/2), U4(t) = U2(at)^2 U2((1-4a)t) U2(at)^2 with
 *     a = 1/(4 - 4^(1/3)) (Sec. 2).  One Trotter step of order k applies Uk(dt).
 *   - exp(-it H_x) and exp(-it H_y) are evaluated as rotations of every spin to the z axis,
 *     a diagonal phase exp(-it D(b)) and the inverse rotations (Sec. 2, Eqs. Rotations,
 *     Single Spin Rotation, Two-Spin-Operators; Sec. 3).
 *
 * State vectors are caller-owned device memory (for example torch tensors), interleaved
 * (re, im): 16 bytes per amplitude for TS_C128, 8 bytes for TS_C64.  The library never
 * allocates or frees them.  A context owns only its own small device tables.
 *
 * Every function returns a ts_status.  On failure ts_last_error() returns a thread-local
 * message.  No C++ exception crosses the ABI.  A context is not thread-safe.  All device
 * work is enqueued on the given stream (a hipStream_t; NULL = the default stream) and is
 * asynchronous unless stated otherwise.  After a failed ts_evolve the state is unspecified.
 */
#ifndef TSSPIN_H
#define TSSPIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TS_OK = 0,
    TS_EINVAL = -1,        /* bad argument: range, null pointer, NaN, alignment        */
    TS_ENOMEM = -2,        /* device tables or scratch do not fit                       */
    TS_EDEVICE = -3,       /* a HIP runtime call failed; the message names it           */
    TS_EUNSUPPORTED = -4,  /* valid request the library does not implement             */
    TS_ENUMERIC = -5       /* the norm watchdog (ts_set_watchdog) saw the norm drift    */
} ts_status;

typedef enum { TS_C128 = 0, TS_C64 = 1 } ts_dtype;

/* One bond (i, j) with its three couplings J^x, J^y, J^z (Sec. 2, Eq. 1). */
typedef struct {
    int32_t i, j;
    double jx, jy, jz;
} ts_bond;

/*
 * Observables (Sec. 4.2 uses the norm and the magnetisation as accuracy probes; the
 * Loschmidt echo is an overlap).  Values are <psi|O|psi> as one double, except the two
 * overlaps, which are complex and take two doubles (re, im).
 *   TS_OBS_NORM        sum_b |c_b|^2
 *   TS_OBS_SX/SY/SZ    <S^a_i>
 *   TS_OBS_SZSZ        <S^z_i S^z_j>
 *   TS_OBS_MZ          <sum_i S^z_i>
 *   TS_OBS_ENERGY      <H>, H of Sec. 2, Eq. 1 (the context's fields and couplings); the x
 *                      and y terms read the amplitudes their spin flips connect
 *   TS_OBS_OVERLAP_SZ  <bra|S^z_i|ket>
 *   TS_OBS_OVERLAP     <bra|ket> (the Loschmidt echo of Sec. 4.2 is |<psi_0|psi>|^2 after
 *                      a forward and a backward evolution)
 * All values are accumulated in FP64 (also for TS_C64 states); the state is not
 * normalised first.
 */
typedef enum {
    TS_OBS_NORM = 0, TS_OBS_SX = 1, TS_OBS_SY = 2, TS_OBS_SZ = 3, TS_OBS_SZSZ = 4,
    TS_OBS_MZ = 5, TS_OBS_ENERGY = 6, TS_OBS_OVERLAP_SZ = 7, TS_OBS_OVERLAP = 8
} ts_obs_kind;

/*
 * kind, spin indices i (and j for SZSZ).  In ts_evolve, `ket` and `bra` index the psi[]
 * array of evolved vectors (bra is used by the overlaps only); `other` is ignored.
 * In ts_expect, the observable acts on psi and `other` (device pointer, same dtype and
 * length) is the bra of an overlap; ket/bra are ignored.
 */
typedef struct {
    int32_t kind, i, j;
    int32_t ket, bra;
    const void *other;
} ts_observable;

typedef struct ts_ctx ts_ctx;

/*
 * Build a context for an N-spin Hamiltonian (Sec. 2, Eq. 1).
 *   n_spins  1..35.  Calls on TS_C128 states accept up to 34 spins and calls on TS_C64
 *            states up to 35; the limit is checked per call.
 *   bonds    n_bonds entries, 0 <= i, j < n_spins, i != j, finite couplings.  May be NULL
 *            when n_bonds == 0.  Copied; the caller keeps ownership.
 *   fields   NULL (all zero) or n_spins*3 doubles h[j][a], a = x, y, z.  Copied.
 *   out      receives the context.
 * Host-only: no device memory is touched until the first call that takes a stream.
 * Errors: TS_EINVAL (range, i == j, non-finite value, NULL out).
 */
ts_status ts_create(int32_t n_spins, const ts_bond *bonds, int32_t n_bonds,
                    const double *fields, ts_ctx **out);

/* Free the context and its device tables (waits for its pending work). NULL is a no-op. */
ts_status ts_destroy(ts_ctx *ctx);

/*
 * Advance n_psi (1..8) state vectors by nsteps Trotter steps of the given order (1, 2 or 4;
 * Sec. 2) with time step dt (any finite value); the vectors are advanced to each record
 * point together, so overlaps between them can be recorded.  U2 and U4 are palindromic, so
 * for orders 2 and 4 the run with -dt is the exact inverse of the run with dt (the Loschmidt
 * echo of Sec. 4.2); U1 is not, and U1(-dt) is not the inverse of U1(dt).  Long runs are
 * executed as repeated plans of at most 32 steps; this changes results only at rounding
 * level (two half phases at a plan boundary instead of one merged phase).
 *   psi       n_psi device pointers, each 2^N amplitudes of `dtype`, evolved in place.
 *             Alignment: 16 bytes (TS_C128) or 8 bytes (TS_C64).
 *   rec/n_rec observables recorded at steps 0, rec_every, 2*rec_every, ... <= nsteps.
 *   rec_out   device pointer to double[(nsteps/rec_every)+1][slots], slots = sum over rec
 *             of 1 (real kinds) or 2 (the overlaps: re, im).  Caller-owned.  May be
 *             NULL when n_rec == 0.  Accumulated in FP64 for both dtypes.  A single
 *             vector that fits one workgroup's LDS, recorded with real kinds only, runs
 *             every segment and record in one launch (records summed there, in another
 *             order than the separate reductions: they agree to rounding).
 *   stream    hipStream_t or NULL.
 * nsteps == 0 records step 0 only (if asked) and changes nothing.
 * With the norm watchdog on (ts_set_watchdog), the call also synchronises the stream and
 * returns TS_ENUMERIC if a vector's norm drifted beyond the bound; the evolution has then
 * completed and the vectors hold its result.
 * Errors: TS_EINVAL (pointers, alignment, order, non-finite dt, rec indices, n > dtype
 * limit), TS_ENOMEM, TS_EDEVICE, TS_ENUMERIC.
 */
ts_status ts_evolve(ts_ctx *ctx, void *const *psi, int32_t n_psi, ts_dtype dtype, double dt,
                    int64_t nsteps, int32_t order, const ts_observable *rec, int32_t n_rec,
                    int32_t rec_every, double *rec_out, void *stream);

/*
 * Norm watchdog of ts_evolve.  Every partial evolution of the Trotter product is unitary
 * (Sec. 2), so the norm of an evolved vector stays constant up to rounding; Sec. 4.2 uses
 * its conservation (and that of the magnetisation) as an accuracy probe.  max_drift < 0
 * (the default) turns the watchdog off.  With max_drift >= 0, every ts_evolve on this
 * context computes the FP64 norm N0 of each vector before the evolution and N1 after it
 * (two reductions and one stream synchronisation per call) and returns TS_ENUMERIC, with
 * the vector and both norms in ts_last_error(), when |N1 - N0| > max_drift * N0 or either
 * norm is not finite (a NaN or infinity in the state).  Typical drifts: about 1e-15 per
 * step for TS_C128 and 1e-7 per step for TS_C64.  Host-only.
 * Errors: TS_EINVAL (NULL ctx, NaN max_drift).
 */
ts_status ts_set_watchdog(ts_ctx *ctx, double max_drift);

/*
 * Local time scale of the Hamiltonian (Sec. 2, Eq. SegundoMomento).  The partial
 * evolutions approximate exp(-itH) well only for steps much shorter than
 *     t_loc = [ max_{j,k} ( sum_a (h^a_j / 2)^2 + sum_a (J^a_jk / 4)^2 )^(1/2) ]^(-1),
 * the maximum taken over every spin j and every spin k bonded to it (no k, J = 0, for a
 * spin without bonds); bonds listed twice count with their summed couplings.  Writes
 * t_loc to *bound (+infinity when H = 0); callers compare dt with it.  Host-only.
 * Errors: TS_EINVAL (NULL pointer).
 */
ts_status ts_dt_bound(ts_ctx *ctx, double *bound);

/*
 * Evaluate n_obs observables of one state psi (device pointer) into out_host (host
 * array of `slots` doubles, laid out as for ts_evolve).  Synchronises the stream.
 * Errors: TS_EINVAL, TS_EDEVICE.
 */
ts_status ts_expect(ts_ctx *ctx, const void *psi, ts_dtype dtype, const ts_observable *obs,
                    int32_t n_obs, double *out_host, void *stream);

/*
 * ts_expect without any allocation, for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid it.  The same
 * observables and values as ts_expect (bit for bit), except TS_OBS_ENERGY
 * (TS_EUNSUPPORTED: it needs the context's device copy of H), written as `slots` doubles
 * to out_dev (device memory, caller-owned), asynchronously on `stream`; it does not
 * synchronise.  The reduction's per-workgroup partials live in a fixed array of 256 KiB
 * (1024 workgroups x 32 doubles) that the library keeps on every GPU it runs on until the
 * process ends, shared by every call on that GPU: calls that overlap on one GPU (on
 * different streams or host threads) race, so order them.  Requests beyond that array
 * are refused with TS_EINVAL (the reduction of any state and up to 16 observables fits).
 * No hipMalloc, hipFree or allocating library call is made.
 * Errors: TS_EINVAL, TS_EUNSUPPORTED, TS_EDEVICE.
 */
ts_status ts_expect_noalloc(ts_ctx *ctx, const void *psi, ts_dtype dtype, const ts_observable *obs,
                            int32_t n_obs, double *out_dev, void *stream);

/*
 * Loss L = <psi(T)|O|psi(T)> of the evolution psi(T) = Uk(dt)^nsteps psi0 (Sec. 2) and its
 * gradient with respect to every coupling and field of Eq. 1, by the adjoint method.  The
 * Trotter product is unitary, so running its partial evolutions in reverse order with -tau
 * undoes the forward run exactly (the Loschmidt-echo property of Sec. 4.2, for every
 * order): the reverse pass recomputes every intermediate state instead of storing them.
 * For each partial evolution
 * G = V exp(-i tau D_a) V^dagger and parameter theta of axis a with weight f_theta(b)
 * (s_j for h^a_j, s_i s_j for J^a_ij):
 *     dL/dtheta += 2 tau sum_b f_theta(b) Im(conj(mu_b) phi_b),
 * mu, phi = the adjoint and forward states in the frame of that partial evolution.  The
 * phase terms commute, so a partial evolution may be applied spin by spin and bond by bond
 * (the light-cone form of ts_cone_describe, used for the reverse pass where it fits): each
 * term's sum is then taken in the frame where that term is applied.  The gradient sums are
 * accumulated in FP64 in an order that may differ from run to run (atomic adds), so the
 * gradient can differ between runs in its last bits; the loss does not.
 *   psi0        device, 2^N amplitudes of dtype; not modified.
 *   loss_obs    one Hermitian observable: TS_OBS_SX, SY, SZ, SZSZ, MZ or ENERGY (ket/bra/
 *               other ignored).  H depends on the parameters, so for TS_OBS_ENERGY every
 *               derivative also gets <psi(T)|dH/dtheta|psi(T)>: <S^a_j> for h^a_j and
 *               <S^a_i S^a_j> for J^a_ij.
 *   loss        host double.
 *   grad_bonds  host double[n_bonds][3] in the order bonds were given to ts_create (a bond
 *               listed twice gets the gradient of the summed coupling in both rows); may be
 *               NULL when there are no bonds.
 *   grad_fields host double[n_spins][3].
 *   workspace   device, caller-owned, 2 * 2^N amplitudes of dtype (overwritten).
 * Systems of fewer than 8 spins run as the same problem on 8 spins (the added spins
 * have no field and no bond, so the result is unchanged); the library then uses a small
 * buffer of its own (3 * 2^8 amplitudes) instead of the workspace.  Synchronises the stream.
 * Errors: TS_EINVAL, TS_ENOMEM, TS_EDEVICE.
 */
ts_status ts_adjoint(ts_ctx *ctx, const void *psi0, ts_dtype dtype, double dt, int64_t nsteps,
                     int32_t order, const ts_observable *loss_obs, double *loss,
                     double *grad_bonds, double *grad_fields, void *workspace, void *stream);

/*
 * Batch of independent systems (for example disorder realisations or random-phase
 * typicality states, Appendix A) evolved together.
 *   n_chains   number of systems.
 *   n_spins    [n_chains] spins of each system (1..35).
 *   bonds      all bonds, system c owning bonds[bond_off[c] .. bond_off[c+1]).
 *   bond_off   [n_chains + 1], bond_off[0] = 0, non-decreasing.
 *   fields     NULL or the concatenated h[n_spins[c]][3] of every system.
 * Host-only.  Errors: TS_EINVAL (per-system messages name the system).
 */
ts_status ts_create_batch(int32_t n_chains, const int32_t *n_spins, const ts_bond *bonds,
                          const int32_t *bond_off, const double *fields, ts_ctx **out);

/*
 * Advance every system of a batch context by nsteps steps (as ts_evolve).  System c's state
 * lives at psi_packed + psi_off[c] amplitudes (device, dtype, caller-owned, in place).
 * Observables (NORM, SX, SY, SZ, SZSZ, MZ; not ENERGY or overlaps; ket/bra ignored) are recorded at
 * steps 0, rec_every, ... into rec_out (device) laid out [n_chains][nsteps/rec_every + 1]
 * [n_rec].  Systems of equal size share one plan: the ones that fit a tile run their whole
 * evolution in one LDS-resident launch (one workgroup per system), the others run one
 * launch per sweep for all systems of that size, each size class on its own stream.  The
 * first call with a given set of arguments captures everything into one hipGraph; calls
 * with the same arguments replay it (the context keeps the 8 most recently used such
 * programs).  If the capture fails, the same launches run uncaptured, in order, on
 * `stream` (ts_batch_stats counts both).  Asynchronous on `stream`.
 * Errors: TS_EINVAL, TS_ENOMEM, TS_EDEVICE.
 */
ts_status ts_evolve_batch(ts_ctx *ctx, void *psi_packed, const int64_t *psi_off, ts_dtype dtype,
                          double dt, int64_t nsteps, int32_t order, const ts_observable *rec,
                          int32_t n_rec, int32_t rec_every, double *rec_out, void *stream);

/*
 * Host-only counters of a batch context's ts_evolve_batch calls, into stats[4]:
 * [0] calls that replayed a captured hipGraph, [1] calls that ran the launches uncaptured
 * because the capture had failed, [2] failed captures, [3] captured programs currently
 * kept.  Errors: TS_EINVAL (NULL pointer).
 */
ts_status ts_batch_stats(ts_ctx *ctx, int64_t *stats);

/*
 * Tile width in bits (2^T amplitudes staged per workgroup) that ts_evolve uses for
 * `dtype` on this context: 8..13 for TS_C128, 8..14 for TS_C64; 0 restores the default
 * (12 for both: 64 KiB (complex128) or 32 KiB (complex64) of LDS per workgroup, so two or
 * more workgroups share a CU and overlap memory with arithmetic).  Narrower tiles cut the
 * state into more bit groups (the closed sets of Sec. 3.3) and can cost more passes;
 * wider ones allow fewer workgroups per CU.  ts_autotune picks per size.
 * Host-only.  Errors: TS_EINVAL.
 */
ts_status ts_set_tile_bits(ts_ctx *ctx, ts_dtype dtype, int32_t tile_bits);

/*
 * Autotuner.  There is no single best tile width, run width or kernel for every size; the
 * paper searched them by brute force per system size and kept the results in a file
 * (Sec. 3.4).  ts_autotune times every candidate (tile width T, register window RB, and
 * the kernel variant) on one Trotter step of this context's system, keeps the fastest
 * for `dtype` on the context, and stores it in a JSON cache (path: $TSSPIN_TUNE_CACHE, else
 * ~/.cache/tsspin/tune.json) keyed by (GPU architecture, n_spins, dtype, order).  Any later
 * context of the same size consults the cache on its first evolution (unless
 * ts_set_tile_bits fixed the width or $TSSPIN_NO_TUNE_CACHE is set).  A missing or damaged
 * cache is ignored.
 * A batch context (ts_create_batch) is tuned as a whole: one step of every system, for
 * each tile width and register window, replayed as the batch's graph; the best is kept on
 * the context (not in the cache file), and use_cache is ignored.
 *   scratch      device, 2^N amplitudes of dtype (a batch: sum over systems of 2^n_c,
 *                packed), overwritten with meaningless values.
 *   use_cache    non-zero: take a cached entry for this key instead of timing, if present.
 *   ms_per_step  NULL or receives the chosen configuration's time per step.
 * Synchronises the stream.  Errors: TS_EINVAL, TS_EDEVICE, TS_ENOMEM.
 */
ts_status ts_autotune(ts_ctx *ctx, ts_dtype dtype, int32_t order, void *scratch, int32_t use_cache,
                      double *ms_per_step, void *stream);

/*
 * The kernel configuration ts_evolve will use for dtype and order: tile width, register
 * window width, and variant (0 register-window sweep, one tile per workgroup; 1 LDS-staged
 * sweep; 2 pipelined register-window sweep, resident workgroups that prefetch their next
 * tile; 3 register-window sweep that runs the sweeps on the top bit group with a
 * complex128 kernel using half the LDS per workgroup, the default for TS_C128, where
 * tiles of 2^11 or 2^12 amplitudes allow it; 4 the light-cone sweeps where the cost model
 * prefers them, else 3 (TS_C128) or 0; 5 register-window sweep whose phase step reads the
 * energies D_a(b) from tables in device memory, one per axis with 2^N doubles (TS_C128)
 * or floats (TS_C64), built once per context: the precomputed-phase mode of Sec. 3.1).
 * Consults the tuning cache like a first evolution does.  Host-only apart from reading the
 * device name.
 */
ts_status ts_get_kernel_config(ts_ctx *ctx, ts_dtype dtype, int32_t order, int32_t *tile_bits,
                               int32_t *reg_bits, int32_t *variant);

/* Thread-local text of the last failure on this thread ("" if none). */
const char *ts_last_error(void);

/*
 * Host-only introspection of the sweep plan ts_evolve would run for one recording
 * segment of `nsteps` steps (the whole run when not recording), for tests and tools.
 * Writes up to `cap` records of 16 int64 each into `out` (may be NULL to query the
 * count) and stores the number of sweeps in *n_sweeps:
 *   [0] tile mask (global bits resident in one workgroup tile)
 *   [1] pre mask  (global bits rotated before the diagonal)
 *   [2] post mask (global bits rotated after the diagonal)
 *   [3] diagonal axis (0 x, 1 y, 2 z, 3 identity phase, -1 none)
 *   [4] quarter-turn count c of the phase factor i^(c*popcount(b)) (0..3)
 *   [5] power-of-two exponent e of the magnitude factor 2^-e
 *   [6] 1 if the magnitude factor also carries 1/sqrt(2)
 *   [7] global phase of the diagonal in eighth turns (0..7)
 *   [8] tile bits T
 *   [9] group index
 *  [10] bit pattern of tau (IEEE-754 binary64)
 *  [11] reserved, 0
 *  [12] register-window width RB of the sweep kernel for this dtype (0 for a plan that
 *       runs in the whole-state kernel)
 *  [13] load window | store window << 8 | (phase window + 1) << 16 | stage count << 24
 *       | LDS transposes << 32 (windows are the lowest tile bit of a window of RB bits)
 *  [14],[15] the stage program, 9 bits per stage from bit 0, seven stages per word:
 *       window (4 bits) | kind << 4 (0 butterflies, 1 phase step) | butterfly mask << 5
 *       (bit v of the mask = tile bit window + v; tile bit k is the k-th lowest set bit
 *       of the tile mask)
 * Every rotation is the unnormalised two-point butterfly (u, v) -> (u + v, u - v) on
 * each listed bit; the diagonal multiplies c_b by
 *     2^-e (1/sqrt2)^[6] exp(i*(pi/4)*[7]) i^(c*popcount(b)) exp(-i*tau*D_axis(b)).
 * tile_bits <= 0 selects the library default for the dtype.
 * Errors: TS_EINVAL.
 */
ts_status ts_plan_describe(ts_ctx *ctx, ts_dtype dtype, double dt, int64_t nsteps,
                           int32_t order, int32_t tile_bits, int64_t *out, int64_t cap,
                           int64_t *n_sweeps);

/*
 * Host-only introspection of the light-cone form of the same segment (for tests and
 * tools).  Operations on different spins commute, so a spin may run several layers ahead
 * of spins it is not coupled to; a light-cone sweep over a window of T spins advances the
 * middle of the window by as many layers as the spins just outside it allow.  The same
 * arithmetic as the plan of ts_plan_describe, regrouped: each layer's butterflies and each
 * phase step's terms are split by spin (field and quarter turn of a spin, one term per
 * bond), and every part runs exactly once.
 * low_bits (<= 0: the library default, 4) memory bits stay in every tile; max_adv (<= 0: no
 * bound) bounds the layers a spin takes in one sweep.  Writes up to `cap` rows of 10 int64
 * into `out` (may be NULL to query the count), stores the row count in *n_rows, and stores
 * in *used (may be NULL) 1 if ts_evolve would run this form for the dtype, else 0:
 *   sweep      [1, window spin mask, spins at memory bits 0..low_bits-1 when loading (mask),
 *               the same when storing, 1 if the store permutes the tile's memory bits,
 *               operation rows that follow, stage count, LDS transposes, 0, 0]
 *   tile bit   [4, tile bit i, spin held, memory bit when loading, memory bit when storing,
 *               0, 0, 0, 0, 0]   (T rows after each sweep row)
 *   stage      [5, register window (its lowest tile bit), 1 if the stage ends with a phase
 *               step, butterfly mask over the window's bits, phase step index, 0, ...]
 *               (the kernel's stage program, after the tile rows; framed by
 *               [5, -1, 0, 0, -1, load window, 0, ...] and [5, -2, 0, 0, -1, store window,
 *               0, ...]; absent where the sweep has no stage program)
 *   butterfly  [2, spin mask, 0, ...]: (u, v) -> (u + v, u - v) on each listed spin's bit
 *   phase step [3, level (index of the folded phase step), spins whose field and quarter
 *               turn apply (mask), bonds whose term applies (mask over the merged bond list
 *               in input order of first appearance; -1 if there are more than 63 bonds),
 *               h, e8, axis, quarter-turn count c, bit pattern of tau, register window of
 *               the step in the kernel (lowest tile bit; -1 if no stage program)]
 *               multiplies c_b by (1/sqrt2)^h exp(i*(pi/4)*e8)
 *               * prod_{q in spins} i^(c*b_q) exp(-i tau h^axis_q s_q)
 *               * prod_{(p,q) in bonds} exp(-i tau J^axis_pq s_p s_q),  s = bit - 1/2.
 * The sweeps start and end with every spin at its own memory bit.
 * Errors: TS_EINVAL (also when no light-cone plan exists for these sizes).
 */
ts_status ts_cone_describe(ts_ctx *ctx, ts_dtype dtype, double dt, int64_t nsteps,
                           int32_t order, int32_t tile_bits, int32_t low_bits, int32_t max_adv,
                           int64_t *out, int64_t cap, int64_t *n_rows, int32_t *used);

#ifdef __cplusplus
}
#endif

#endif /* TSSPIN_H */

// kernels.hip -- gfx950 device code of libtsspin.
//
// Kernel families:
//   sweep_reg_kernel   one pass over a state larger than a tile.  Each workgroup owns one
//                      closed set of 2^T amplitudes (Sec. 3.3: fixing the spins outside a
//                      group of bits leaves a set closed under flipping the spins inside it)
//                      and runs a host-planned stage program on it: butterflies on the
//                      bits of one layer, the phase step, butterflies of the next layer.
//                      Each thread holds 2^RB amplitudes along a window of RB tile bits in
//                      registers; changing window is one transpose through LDS.  The low
//                      index bits always stay in the tile, so every workgroup moves
//                      contiguous runs (Sec. 3.4), and the phase is fused with the rotations
//                      (Sec. 3.1).
//   sweep_pipe_kernel  the same stages with a grid of resident workgroups that prefetch
//                      their next tile into a second register set.
//   sweep_kernel       the same pass with the tile staged in LDS (kept for tuning).
//   resident_kernel    a state that fits one tile: a whole recording segment in LDS, one
//                      workgroup per state (or per chain of a batch).
//   reduce_kernel, batch_reduce_kernel, finalize_kernel
//                      FP64 observables of Sec. 4.2 (norm, spin components, correlations,
//                      magnetisation, overlaps) and the energy <H> of Eq. 1, with a
//                      fixed-order compensated final sum.
//   apply_obs_kernel, apply_ham_kernel, grad_reduce_kernel
//                      the adjoint: lambda = O psi (O = H for the energy), and the gradient
//                      sums in a phase frame.
//
// Phase step.  The energy of axis a is D(b) = sum_j h_j s_j + sum_(i,j) J_ij s_i s_j with
// s = +-1/2 (Sec. 2, Eqs. 1 and ZZ-Phases).  It is split by who fixes which bits:
//   workgroup  the bits outside the tile: a host table holds per tile the phase factors of
//              the outside energy and of the effective field on each tile bit;
//   thread     the tile bits outside its register window: a host table per thread pattern
//              holds the pair phases among them and the fields they put on window bits;
//   element    a Gray-code walk over the window bits times a table of the couplings
//              inside the window.
// Every phase argument and phase factor is FP64 for both storage precisions.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "kernels.hpp"

namespace tsk {

template <typename R> struct Vec;
template <> struct Vec<double> { using T = double2; };
template <> struct Vec<float> { using T = float2; };

constexpr int kThreads = 256;
constexpr int kFixedBits = 8;  // log2(kThreads): tile bits fixed per thread

__device__ __forceinline__ uint64_t dep(uint64_t x, const Run *r, int n)
{
    uint64_t out = 0;
    for (int i = 0; i < n; ++i) out |= ((x >> r[i].src) & ((1ull << r[i].len) - 1ull)) << r[i].dst;
    return out;
}

// insert a zero bit at position k
__device__ __forceinline__ uint32_t ins0(uint32_t g, int k)
{
    return ((g >> k) << (k + 1)) | (g & ((1u << k) - 1u));
}

template <typename V>
__device__ __forceinline__ void bfly(V &a, V &b)
{
    V u = a, v = b;
    a.x = u.x + v.x;
    a.y = u.y + v.y;
    b.x = u.x - v.x;
    b.y = u.y - v.y;
}

// Walsh-Hadamard butterflies on 1, 2 or 3 tile bits over the LDS tile of ne amplitudes.
template <typename V>
__device__ void wht_pass(V *tile, int ne, int nk, int k0, int k1, int k2)
{
    if (nk == 3) {
        const int ng = ne >> 3;
        const uint32_t d0 = 1u << k0, d1 = 1u << k1, d2 = 1u << k2;
        for (int g = threadIdx.x; g < ng; g += kThreads) {
            const uint32_t t = ins0(ins0(ins0((uint32_t)g, k0), k1), k2);
            V x[8];
#pragma unroll
            for (int i = 0; i < 8; ++i)
                x[i] = tile[t + ((i & 1) ? d0 : 0) + ((i & 2) ? d1 : 0) + ((i & 4) ? d2 : 0)];
#pragma unroll
            for (int s = 1; s < 8; s <<= 1)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (!(i & s)) bfly(x[i], x[i + s]);
#pragma unroll
            for (int i = 0; i < 8; ++i)
                tile[t + ((i & 1) ? d0 : 0) + ((i & 2) ? d1 : 0) + ((i & 4) ? d2 : 0)] = x[i];
        }
    } else if (nk == 2) {
        const int ng = ne >> 2;
        const uint32_t d0 = 1u << k0, d1 = 1u << k1;
        for (int g = threadIdx.x; g < ng; g += kThreads) {
            const uint32_t t = ins0(ins0((uint32_t)g, k0), k1);
            V x0 = tile[t], x1 = tile[t + d0], x2 = tile[t + d1], x3 = tile[t + d0 + d1];
            bfly(x0, x1);
            bfly(x2, x3);
            bfly(x0, x2);
            bfly(x1, x3);
            tile[t] = x0;
            tile[t + d0] = x1;
            tile[t + d1] = x2;
            tile[t + d0 + d1] = x3;
        }
    } else {
        const int ng = ne >> 1;
        const uint32_t d0 = 1u << k0;
        for (int g = threadIdx.x; g < ng; g += kThreads) {
            const uint32_t t = ins0((uint32_t)g, k0);
            V x0 = tile[t], x1 = tile[t + d0];
            bfly(x0, x1);
            tile[t] = x0;
            tile[t + d0] = x1;
        }
    }
}

// All butterflies of a layer restricted to the tile bits in `mask`, three bits per pass.
template <typename V>
__device__ void wht_layer(V *tile, int ne, uint32_t mask)
{
    while (mask) {
        int k[3] = {0, 0, 0};
        int nk = 0;
        while (mask && nk < 3) {
            k[nk++] = __builtin_ctz(mask);
            mask &= mask - 1;
        }
        wht_pass(tile, ne, nk, k[0], k[1], k[2]);
        __syncthreads();
    }
}

// Complex products with explicit FMAs: the rounding is then the same in every kernel,
// whatever the compiler would otherwise contract in the surrounding code.
__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(__builtin_fma(a.x, b.x, -(a.y * b.y)), __builtin_fma(a.x, b.y, a.y * b.x));
}

// multiply by i^m
__device__ __forceinline__ double2 qturn(double2 a, int m)
{
    switch (m & 3) {
    case 1: return make_double2(-a.y, a.x);
    case 2: return make_double2(-a.x, -a.y);
    case 3: return make_double2(a.y, -a.x);
    default: return a;
    }
}

__device__ __forceinline__ double2 expi(double phi)
{
    double s, c;
    sincos(phi, &s, &c);
    return make_double2(c, s);
}

// complex64: the product with the FP64 factor is formed in FP64 and rounded once.  Rounding
// the factor to FP32 first would give it a modulus 1 + O(2^-24) that every amplitude sharing
// it picks up alike: a systematic drift of the norm (about 3e-7 per fourth-order step in the
// Loschmidt echo of a 14-spin ring), where one rounding of each product leaves only
// independent errors.
__device__ __forceinline__ void apply_phase(double2 &x, double2 z) { x = cmul(x, z); }
__device__ __forceinline__ void apply_phase(float2 &x, double2 z)
{
    const double xr = x.x, xi = x.y;
    x.x = (float)__builtin_fma(xr, z.x, -(xi * z.y));
    x.y = (float)__builtin_fma(xr, z.y, xi * z.x);
}

// Per-launch table over the var bits: i^(c*popcount(j)) * exp(-i tau Q(j)), Q = the
// couplings among var bits (tile bits 8..T-1).  Built by threads j < 2^V.
template <int T>
__device__ void build_qtab(double2 *qtab, const DiagArgs &d, const double *jt)
{
    constexpr int V = (T > kFixedBits) ? T - kFixedBits : 0;
    const int j = threadIdx.x;
    if (j < (1 << V)) {
        double q = 0.0;
        if (d.axis < 3) {
#pragma unroll
            for (int v1 = 0; v1 < V; ++v1)
#pragma unroll
                for (int v2 = v1 + 1; v2 < V; ++v2) {
                    const double c = jt[(kFixedBits + v1) * T + kFixedBits + v2];
                    const double s = (((j >> v1) ^ (j >> v2)) & 1) ? -0.25 : 0.25;
                    q += c * s;
                }
        }
        qtab[j] = qturn(expi(-d.tau * q), d.qturn * __builtin_popcount(j));
    }
}

// Phase step on the thread's 2^(T-8) amplitudes t = tid + 256*j of the LDS tile.
// wg = [C, geff_0 .. geff_{T-1}] of this workgroup, jt = tile couplings (upper triangle),
// b_thread = global index of element j = 0.
template <int T, typename V>
__device__ void diag_step(V *tile, int ne, const DiagArgs &d, const double *wg, const double *jt,
                          const double2 *qtab, uint64_t b_thread)
{
    constexpr int NV = (T > kFixedBits) ? T - kFixedBits : 0;
    constexpr int EPT = 1 << NV;
    constexpr int FB = (T < kFixedBits) ? T : kFixedBits;
    const int tid = threadIdx.x;
    if (tid >= ne) return;
    double C = 0.0;
    double g[NV > 0 ? NV : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) g[v] = 0.0;
    if (d.axis < 3) {
        C = wg[0];
#pragma unroll
        for (int k = 0; k < FB; ++k) C += (((tid >> k) & 1) ? 0.5 : -0.5) * wg[1 + k];
#pragma unroll
        for (int k1 = 0; k1 < FB; ++k1)
#pragma unroll
            for (int k2 = k1 + 1; k2 < FB; ++k2)
                C += jt[k1 * T + k2] * ((((tid >> k1) ^ (tid >> k2)) & 1) ? -0.25 : 0.25);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            double gv = wg[1 + kFixedBits + v];
#pragma unroll
            for (int k = 0; k < kFixedBits; ++k)
                gv += jt[k * T + kFixedBits + v] * (((tid >> k) & 1) ? 0.5 : -0.5);
            g[v] = gv;
        }
    }
    // energy of element j = 0 (all var bits down) without the var-var part (in qtab)
    double e0 = C;
#pragma unroll
    for (int v = 0; v < NV; ++v) e0 -= 0.5 * g[v];
    double2 p = cmul(make_double2(d.kre, d.kim), expi(-d.tau * e0));
    p = qturn(p, d.qturn * __popcll(b_thread));
    double2 w[NV > 0 ? NV : 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) w[v] = expi(-d.tau * g[v]);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
        const int j = k ^ (k >> 1);
        if (k > 0) {
            const int v = __builtin_ctz(k);
            const double2 wv = ((j >> v) & 1) ? w[v] : make_double2(w[v].x, -w[v].y);
            p = cmul(p, wv);
        }
        const double2 z = cmul(p, qtab[j]);
        V x = tile[tid + kThreads * j];
        apply_phase(x, z);
        tile[tid + kThreads * j] = x;
    }
}

template <typename R, int T>
__global__ __launch_bounds__(kThreads) void sweep_kernel(typename Vec<R>::T *__restrict__ psi,
                                                         SweepArgs a)
{
    using V = typename Vec<R>::T;
    constexpr int NE = 1 << T;
    constexpr int EPT = NE / kThreads;
    constexpr int NV = T - kFixedBits;
    __shared__ V tile[NE];
    __shared__ double2 qtab[1 << NV];
    const int tid = threadIdx.x;
    const uint64_t base = dep(blockIdx.x, a.out_runs, a.n_out_runs);
    const uint64_t bt = base | dep((uint64_t)tid, a.tile_runs, a.n_tile_runs);
    {
        V r[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            r[j] = psi[bt | dep((uint64_t)j << kFixedBits, a.tile_runs, a.n_tile_runs)];
#pragma unroll
        for (int j = 0; j < EPT; ++j) tile[tid + kThreads * j] = r[j];
    }
    if (a.d.axis >= 0) build_qtab<T>(qtab, a.d, a.jt);
    __syncthreads();
    wht_layer(tile, NE, a.pre_mask);
    if (a.d.axis >= 0) {
        const double *wg = (a.d.axis < 3) ? a.wg + (size_t)blockIdx.x * (T + 1) : nullptr;
        diag_step<T>(tile, NE, a.d, wg, a.jt, qtab, bt);
        __syncthreads();
    }
    wht_layer(tile, NE, a.post_mask);
    {
        V r[EPT];
#pragma unroll
        for (int j = 0; j < EPT; ++j) r[j] = tile[tid + kThreads * j];
#pragma unroll
        for (int j = 0; j < EPT; ++j)
            psi[bt | dep((uint64_t)j << kFixedBits, a.tile_runs, a.n_tile_runs)] = r[j];
    }
}

// --------------------------------------------------------- register-window sweep
//
// Each of the 2^(T-RB) threads holds 2^RB amplitudes of the tile in registers: the ones
// whose tile indices differ only in a window of RB consecutive tile bits [w, w+RB).
// Butterflies on window bits need no LDS; moving to another window is one transpose
// through a padded LDS buffer.  The stage list (window, butterfly mask, phase step) is
// planned on the host; loads and stores use windows that keep the low index bits on the
// lanes, so every wavefront instruction moves whole 128-byte lines.

// tile index of element r = 0 of thread tid in the layout with window w
template <int RB>
__device__ __forceinline__ uint32_t thread_part(uint32_t tid, int w)
{
    return (tid & ((1u << w) - 1u)) | ((tid >> w) << (w + RB));
}

__device__ __forceinline__ uint32_t lds_pos(uint32_t t) { return t + (t >> 4); }

template <int RB, typename V>
__device__ __forceinline__ void reg_bfly(V (&x)[1 << RB], uint32_t mask)
{
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        if (!((mask >> v) & 1u)) continue;
#pragma unroll
        for (int r = 0; r < (1 << RB); ++r)
            if (!(r & (1 << v))) bfly(x[r], x[r | (1 << v)]);
    }
}

// Workgroup barrier that orders LDS traffic only: it waits for this wave's LDS operations
// (lgkmcnt) but not for its outstanding global loads, so prefetches stay in flight.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

template <int RB, typename V>
__device__ __forceinline__ void reg_transpose(V (&x)[1 << RB], V *lds, int from, int to)
{
    const uint32_t tid = threadIdx.x;
    lds_barrier();
    const uint32_t tf = thread_part<RB>(tid, from);
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) lds[lds_pos(tf | ((uint32_t)r << from))] = x[r];
    lds_barrier();
    const uint32_t tt = thread_part<RB>(tid, to);
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r] = lds[lds_pos(tt | ((uint32_t)r << to))];
}

// The same transpose for complex128 through an LDS buffer of doubles: real parts first,
// then imaginary parts.  Half the LDS of reg_transpose, at the cost of two more barriers.
template <int RB>
__device__ __forceinline__ void reg_transpose_half(double2 (&x)[1 << RB], double *lds, int from, int to)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t tf = thread_part<RB>(tid, from);
    const uint32_t tt = thread_part<RB>(tid, to);
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) lds[lds_pos(tf | ((uint32_t)r << from))] = x[r].x;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r].x = lds[lds_pos(tt | ((uint32_t)r << to))];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) lds[lds_pos(tf | ((uint32_t)r << from))] = x[r].y;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r].y = lds[lds_pos(tt | ((uint32_t)r << to))];
}

template <int RB, typename V>
__device__ __forceinline__ void any_transpose(V (&x)[1 << RB], V *lds, int from, int to)
{
    reg_transpose<RB>(x, lds, from, to);
}
template <int RB>
__device__ __forceinline__ void any_transpose(double2 (&x)[1 << RB], double *lds, int from, int to)
{
    reg_transpose_half<RB>(x, lds, from, to);
}

// A read-only table whose entries every lane reads at the same address: through the
// constant address space the loads become scalar loads into SGPRs, which the complex
// products then take as operands (no LDS staging, no LDS reads, no vector registers).
typedef const __attribute__((address_space(4))) double *ctab;
__device__ __forceinline__ ctab as_const(const double *p)
{
    return (ctab)(const __attribute__((address_space(4))) void *)p;
}
__device__ __forceinline__ double2 ld2(ctab t, uint32_t i) { return make_double2(t[2 * i], t[2 * i + 1]); }
// One word of every 64-byte line of the `bytes` bytes at t (L lines at most), through the
// scalar data cache: the table's later scalar loads then hit there.  The lines run from the
// one holding the first byte to the one holding the last (clamped there).
template <int L>
__device__ __forceinline__ uint32_t ctab_touch(ctab t, uint32_t bytes)
{
    typedef const __attribute__((address_space(4))) uint32_t *cword;
    const uint64_t first = (uint64_t)t & ~63ull, last = ((uint64_t)t + bytes - 1) & ~63ull;
    uint32_t acc = 0;
#pragma unroll
    for (int l = 0; l < L; ++l) {
        const uint64_t at = first + 64 * l;
        acc ^= *(cword)(at < last ? at : last);
    }
    return acc;
}

// Streaming access to the state, which a sweep reads and writes once: loads and stores
// with the non-temporal hint (the light-cone sweeps at N = 27 ran 2% faster with it).
__device__ __forceinline__ double2 ntload(const double2 *p)
{
    return make_double2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ float2 ntload(const float2 *p)
{
    return make_float2(__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y));
}
__device__ __forceinline__ void ntstore(double2 *p, double2 v)
{
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}
__device__ __forceinline__ void ntstore(float2 *p, float2 v)
{
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
}

// entry i of a table of (re, im) pairs in LDS or, read with scalar loads, in memory
__device__ __forceinline__ double2 tab2(const double2 *t, uint32_t i) { return t[i]; }
__device__ __forceinline__ double2 tab2(ctab t, uint32_t i) { return ld2(t, i); }
// exp(0) on every entry: the workgroup row of a phase step without energy
__constant__ double kUnitRow[2 * 16] = {1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0,
                                        1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0, 1, 0};

// Workgroup phase factors in LDS: wgf[0] = kappa exp(-i tau C), wgf[1+k] = exp(-i tau geff_k/2)
// for every tile bit k (C, geff: the outside-bit energy and fields of this workgroup).
// Thread k <= T passes entry k of its tile's row of the host factor table ((1, 0) when the
// phase step has no energy).
template <int T>
__device__ __forceinline__ void put_wgf(double2 *wgf, const DiagArgs &d, double2 f)
{
    const int k = threadIdx.x;
    if (k <= T) wgf[k] = k == 0 ? cmul(make_double2(d.kre, d.kim), f) : f;
}

// Phase step on the registers in the layout with window w.  With s = bit - 1/2 and the
// tile bits split into the thread's bits (outside the window) and the window bits v,
//   E = C + sum_thr s_k geff_k + sum_(thr pairs) J s s + sum_v s_v (geff_{w+v} + h_v) + Q(r),
//   h_v = sum_thr J_{k,w+v} s_k,  Q = couplings inside the window,
// so exp(-i tau E) is a product of: the workgroup factors wgf; a host table per thread
// pattern (thread pairs with their quarter turns, and exp(-i tau h_v/2)); and, per element,
// a Gray-code walk over the window bits times the window table q[r].  wgf and q are in LDS
// or read with scalar loads (W, Q); w0 is entry 0 of wgf (with the step's scalar kappa).
template <int T, int RB, typename V, typename W, typename Q>
__device__ void reg_diag_tab(V (&x)[1 << RB], const DiagArgs &d, W wgf, double2 w0,
                             const double2 (&th)[1 + RB], Q q, uint32_t t0, uint64_t base, int w)
{
    double2 p = qturn(cmul(w0, th[0]), d.qturn * __popcll(base));
#pragma unroll
    for (int k = 0; k < T; ++k) {
        if ((unsigned)(k - w) < (unsigned)RB) continue;
        const double2 G = tab2(wgf, 1 + k);
        p = cmul(p, ((t0 >> k) & 1) ? G : make_double2(G.x, -G.y));
    }
    double2 wv[RB];
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        const double2 u = cmul(tab2(wgf, 1 + w + v), th[1 + v]);
        p = cmul(p, make_double2(u.x, -u.y));  // window bits start down: s = -1/2
        wv[v] = cmul(u, u);
    }
#pragma unroll
    for (int k = 0; k < (1 << RB); ++k) {
        const int j = k ^ (k >> 1);
        if (k > 0) {
            const int v = __builtin_ctz(k);
            p = cmul(p, ((j >> v) & 1) ? wv[v] : make_double2(wv[v].x, -wv[v].y));
        }
        apply_phase(x[j], cmul(p, tab2(q, j)));
    }
}

// One tile per workgroup; overlap of memory and ALU comes from the other resident
// workgroups of the CU.  L is the LDS element of the transposes (the amplitude type, or
// double for the half-buffer complex128 variant).
// sin and cos of x for |x| < 2^20 (the host checks the bound), to a few ulp: Cody and
// Waite's reduction by pi/2 (pi/2 = P1 + P2, P1 holding 27 significant bits so that k * P1 is
// exact) to |r| <= pi/4, then the Taylor series of sin r and cos r through r^17 and r^16
// (truncation below 1e-18 there), in Horner form in r^2.  The library sincos carries a
// path for arbitrary arguments whose registers the sweep cannot spare.
__device__ __forceinline__ void sincos_bounded(double x, double *sn, double *cs)
{
    constexpr double P1 = 1.570796325802803, P2 = 9.920935796805404e-10;
    const double k = rint(x * 0.63661977236758134);   // 2 / pi
    double r = __builtin_fma(-k, P1, x);
    r = __builtin_fma(-k, P2, r);
    const double z = r * r;
    double ps = 1.0 / 355687428096000.0;                // 1/17!
    ps = __builtin_fma(ps, z, -1.0 / 1307674368000.0);  // 1/15!
    ps = __builtin_fma(ps, z, 1.0 / 6227020800.0);
    ps = __builtin_fma(ps, z, -1.0 / 39916800.0);
    ps = __builtin_fma(ps, z, 1.0 / 362880.0);
    ps = __builtin_fma(ps, z, -1.0 / 5040.0);
    ps = __builtin_fma(ps, z, 1.0 / 120.0);
    ps = __builtin_fma(ps, z, -1.0 / 6.0);
    const double s0 = __builtin_fma(ps * z, r, r);
    double pc = 1.0 / 20922789888000.0;                 // 1/16!
    pc = __builtin_fma(pc, z, -1.0 / 87178291200.0);    // 1/14!
    pc = __builtin_fma(pc, z, 1.0 / 479001600.0);
    pc = __builtin_fma(pc, z, -1.0 / 3628800.0);
    pc = __builtin_fma(pc, z, 1.0 / 40320.0);
    pc = __builtin_fma(pc, z, -1.0 / 720.0);
    pc = __builtin_fma(pc, z, 1.0 / 24.0);
    pc = __builtin_fma(pc, z, -0.5);
    const double c0 = __builtin_fma(pc, z, 1.0);
    const int q = (int)k & 3;
    *sn = q == 0 ? s0 : q == 1 ? c0 : q == 2 ? -s0 : -c0;
    *cs = q == 0 ? c0 : q == 1 ? -s0 : q == 2 ? -c0 : s0;
}

// Phase step from an energy table: register r holds basis index b = gd | off[r], whose
// energy D_axis(b) is read from HBM; the factor kappa i^(c popcount(b)) exp(-i tau D) is
// formed in FP64 (argument and sin/cos) and applied with one rounding.
template <int RB, typename V, typename ET>
__device__ __forceinline__ void reg_diag_etab(V (&x)[1 << RB], const DiagArgs &d, const ET *et, uint64_t gd,
                                              const uint64_t *off, bool energy)
{
    ET e[1 << RB];
    if (energy) {
#pragma unroll
        for (int r = 0; r < (1 << RB); ++r) e[r] = et[gd | off[r]];
    }
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        double sn = 0.0, cs = 1.0;
        if (energy) sincos_bounded(d.tau * (double)e[r], &sn, &cs);
        const double2 z = qturn(cmul(make_double2(d.kre, d.kim), make_double2(cs, -sn)),
                                d.qturn * __popcll(gd | off[r]));
        apply_phase(x[r], z);
    }
}

template <typename R, int T, int RB, typename L, bool ETAB = false>
__device__ __forceinline__ void reg_sweep(typename Vec<R>::T *__restrict__ psi, const RegSweepArgs &a, L *lds)
{
    using V = typename Vec<R>::T;
    constexpr int E = 1 << RB;
    const uint32_t tid = threadIdx.x;
    uint64_t tile = blockIdx.x;
    const double *wgp = a.wgf;
    const double *dtp = a.dtab;
    if (a.chains) {  // batched: this workgroup's chain
        const uint64_t c = tile / a.tiles_per_chain;
        tile -= c * a.tiles_per_chain;
        const ChainPtrs cp = a.chains[c];
        psi = static_cast<V *>(cp.psi);
        wgp = cp.wgf;
        dtp = cp.dtab;
    } else {
        if (a.psi2 && tile >= a.n_tiles) {  // second state of a pair launch
            psi = static_cast<V *>(a.psi2);
            tile -= a.n_tiles;
        }
        if (a.reverse) tile = a.n_tiles - 1 - tile;
        // Rotated order: workgroups launched together then take tiles spread over the top
        // bits of the tile index instead of neighbouring ones.  A strided tile reads short
        // runs far apart; neighbouring strided tiles read neighbouring runs at the same far
        // offsets.  Spreading them over the address space ran about 5% faster on an 8 GiB
        // state (the host sets rot for large states' strided groups only).
        if (a.rot) {
            const int nb = 63 - __builtin_clzll(a.n_tiles);
            tile = (tile >> a.rot) | ((tile & ((1ull << a.rot) - 1)) << (nb - a.rot));
        }
    }
    const bool has_diag = a.diag_win >= 0;
    const uint64_t base = dep(tile, a.out_runs, a.n_out_runs);
    V x[E];
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a.load_win), a.tile_runs, a.n_tile_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = ntload(&psi[gb | a.load_off[r]]);
    }
    // this thread's row of the host phase table; the workgroup's row of factors (exp(0)
    // everywhere for a step without energy) and the window table, read with scalar loads at
    // the phase step
    double2 th[1 + RB];
    ctab wrow = as_const(kUnitRow), qtab = as_const(kUnitRow);
    if (!ETAB && has_diag) {
        const double2 *dt = reinterpret_cast<const double2 *>(dtp);
#pragma unroll
        for (int v = 0; v <= RB; ++v) th[v] = dt[(size_t)tid * (1 + RB) + v];
        qtab = as_const(dtp) + 2 * ((size_t)1 << (T - RB)) * (1 + RB);
        if (a.d.axis < 3) wrow = as_const(wgp) + 2 * tile * (T + 1);
        // bring both into the scalar cache behind the tile's loads
        const uint32_t t = ctab_touch<((T + 1) * 16 + 63) / 64 + 1>(wrow, 16 * (T + 1)) ^
                           ctab_touch<(16 << RB) / 64>(qtab, 16 << RB);
        asm volatile("" ::"s"(t));
    }
    int cur = a.load_win;
    for (int s = 0; s < a.n_stages; ++s) {
        const uint64_t word = s < kStagesPerWord ? a.st_code[0] : a.st_code[1];
        const uint32_t code = (uint32_t)(word >> (9 * (s % kStagesPerWord))) & 0x1FFu;
        const int w = (int)(code & 15u);
        if (w != cur) {
            any_transpose<RB>(x, lds, cur, w);
            cur = w;
        }
        if (!((code >> 4) & 1u)) {
            reg_bfly<RB>(x, code >> 5);
        } else if constexpr (ETAB) {
            const uint64_t gd = base | dep(thread_part<RB>(tid, w), a.tile_runs, a.n_tile_runs);
            reg_diag_etab<RB>(x, a.d, static_cast<const R *>(a.etab), gd, a.diag_off,
                              a.etab != nullptr && a.d.axis < 3);
        } else {
            const double2 w0 = cmul(make_double2(a.d.kre, a.d.kim), ld2(wrow, 0));
            reg_diag_tab<T, RB>(x, a.d, wrow, w0, th, qtab, thread_part<RB>(tid, w), base, w);
        }
    }
    if (cur != a.store_win) any_transpose<RB>(x, lds, cur, a.store_win);
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a.store_win), a.tile_runs, a.n_tile_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) ntstore(&psi[gb | a.store_off[r]], x[r]);
    }
}

template <typename R, int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void sweep_reg_kernel(typename Vec<R>::T *__restrict__ psi,
                                                                  RegSweepArgs a)
{
    constexpr int NE = 1 << T;
    __shared__ typename Vec<R>::T lds[NE + NE / 16];
    reg_sweep<R, T, RB>(psi, a, lds);
}

// The register-window sweep with the phase step from an energy table in HBM.
template <typename R, int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void sweep_etab_kernel(typename Vec<R>::T *__restrict__ psi,
                                                                   RegSweepArgs a)
{
    constexpr int NE = 1 << T;
    __shared__ typename Vec<R>::T lds[NE + NE / 16];
    reg_sweep<R, T, RB, typename Vec<R>::T, true>(psi, a, lds);
}

// Energy table of one axis: out[b] = sum_i h_i s_i(b) + sum_bonds J s_i(b) s_j(b), the bonds
// read as uniform (scalar) values, each term +-J/4 by the parity of its two bits.
template <typename ET>
__global__ __launch_bounds__(kThreads) void energy_table_kernel(ET *__restrict__ out, int n,
                                                                const double *__restrict__ h,
                                                                const HamBond *__restrict__ bonds, int nb,
                                                                int axis, uint64_t count)
{
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < count;
         b += (uint64_t)gridDim.x * kThreads) {
        double e = 0.0;
        for (int i = 0; i < n; ++i) e += ((b >> i) & 1) ? 0.5 * h[3 * i + axis] : -0.5 * h[3 * i + axis];
        for (int k = 0; k < nb; ++k) {
            const HamBond hb = bonds[k];
            const double J = axis == 0 ? hb.jx : axis == 1 ? hb.jy : hb.jz;
            e += (((b >> hb.i) ^ (b >> hb.j)) & 1) ? -0.25 * J : 0.25 * J;
        }
        out[b] = (ET)e;
    }
}

// ------------------------------------------------------------ adjoint pair sweep
//
// One reverse sweep of the adjoint on psi (x) and lambda (y) in the same workgroup: every
// stage runs on both; the phase step forms each factor once and applies it to both, then
// takes the gradient sums of its axis in registers.  The amplitudes then sit in the frame
// of that phase step, scaled as the split-phase plan would store them, so the sums are the
// ones that plan's separate pass formed.

template <int T, int RB, typename V>
__device__ __forceinline__ void reg_diag_pair(V (&x)[1 << RB], V (&y)[1 << RB], const DiagArgs &d,
                                              const double2 *wgf, const double2 (&th)[1 + RB],
                                              const double2 *q, uint32_t t0, uint64_t base, int w)
{
    double2 p = qturn(cmul(wgf[0], th[0]), d.qturn * __popcll(base));
#pragma unroll
    for (int k = 0; k < T; ++k) {
        if ((unsigned)(k - w) < (unsigned)RB) continue;
        const double2 G = wgf[1 + k];
        p = cmul(p, ((t0 >> k) & 1) ? G : make_double2(G.x, -G.y));
    }
    double2 wv[RB];
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        const double2 u = cmul(wgf[1 + w + v], th[1 + v]);
        p = cmul(p, make_double2(u.x, -u.y));
        wv[v] = cmul(u, u);
    }
#pragma unroll
    for (int k = 0; k < (1 << RB); ++k) {
        const int j = k ^ (k >> 1);
        if (k > 0) {
            const int v = __builtin_ctz(k);
            p = cmul(p, ((j >> v) & 1) ? wv[v] : make_double2(wv[v].x, -wv[v].y));
        }
        const double2 z = cmul(p, q[j]);
        apply_phase(x[j], z);
        apply_phase(y[j], z);
    }
}

// Gradient sums of one phase step from the registers of the window w: per thread the Walsh
// sums M[m] of w_j = Im(conj(y_j) x_j) over the subsets m of the window bits; each wave's
// lanes then take one parameter each and sum its sign times M over the wave's 64 lanes
// (through LDS), and one thread per parameter adds the workgroup's total to its slot.
// gm holds [waves][16][65] doubles, red [waves][64].
template <int T, int RB, typename V>
__device__ __forceinline__ void pair_grad(const V (&x)[1 << RB], const V (&y)[1 << RB], const PairGradArgs &g,
                                          uint64_t base, int w, double *gm, double *red)
{
    constexpr int E = 1 << RB;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    constexpr int NW = (1 << (T - RB)) / 64 > 0 ? (1 << (T - RB)) / 64 : 1;
    constexpr int WL = (1 << (T - RB)) < 64 ? (1 << (T - RB)) : 64;   // threads per wave
    double M[E];
#pragma unroll
    for (int j = 0; j < E; ++j) M[j] = (double)y[j].x * (double)x[j].y - (double)y[j].y * (double)x[j].x;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (!(j & (1 << k))) {
                const double w0 = M[j], w1 = M[j | (1 << k)];
                M[j] = w0 + w1;
                M[j | (1 << k)] = 0.5 * (w1 - w0);
            }
    lds_barrier();   // the transpose buffer is free: every wave is past its last transpose
    double *gw = gm + (size_t)wave * (E * 65);
#pragma unroll
    for (int m = 0; m < E; ++m) gw[m * 65 + lane] = M[m];
    lds_barrier();
    const uint32_t wbase = wave * 64u;
    for (int p0 = 0; p0 < g.np; p0 += WL) {
        const int p = p0 + (int)lane;
        double acc = 0.0;
        if (p < g.np) {
            const int i = g.pi[p], j = g.pj[p];
            int m = 0, ki = -1, kj = -1;
            double s = 1.0;
            const int bi = g.tile_bit[i];
            if (bi < 0) s = ((base >> i) & 1) ? 0.5 : -0.5;
            else if ((unsigned)(bi - w) < (unsigned)RB) m |= 1 << (bi - w);
            else ki = bi;
            if (j >= 0) {
                const int bj = g.tile_bit[j];
                if (bj < 0) s *= ((base >> j) & 1) ? 0.5 : -0.5;
                else if ((unsigned)(bj - w) < (unsigned)RB) m |= 1 << (bj - w);
                else kj = bj;
            }
            for (int t = 0; t < WL; ++t) {
                const uint32_t tp = thread_part<RB>(wbase + (uint32_t)t, w);
                double f = gw[m * 65 + t];
                if (ki >= 0) f *= ((tp >> ki) & 1) ? 0.5 : -0.5;
                if (kj >= 0) f *= ((tp >> kj) & 1) ? 0.5 : -0.5;
                acc += f;
            }
            acc *= s;
        }
        red[wave * 64 + lane] = acc;
        lds_barrier();
        if (wave == 0 && p < g.np) {
            double tot = 0.0;
            for (int v = 0; v < NW; ++v) tot += red[v * 64 + lane];
            g.slots[(size_t)blockIdx.x * g.stride + g.off + g.col[p]] += g.coef * tot;
        }
        lds_barrier();
    }
}

template <typename R, int T, int RB, typename L>
__device__ __forceinline__ void reg_sweep_pair(typename Vec<R>::T *__restrict__ psi, typename Vec<R>::T *__restrict__ lam,
                                               const RegSweepArgs &a, const PairGradArgs &g, L *lds,
                                               double2 *wgf, double2 *q, double *red)
{
    using V = typename Vec<R>::T;
    constexpr int E = 1 << RB;
    const uint32_t tid = threadIdx.x;
    uint64_t tile = blockIdx.x;
    if (a.reverse) tile = a.n_tiles - 1 - tile;
    const bool has_diag = a.diag_win >= 0;
    const uint64_t base = dep(tile, a.out_runs, a.n_out_runs);
    V x[E], y[E];
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a.load_win), a.tile_runs, a.n_tile_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            x[r] = psi[gb | a.load_off[r]];
            y[r] = lam[gb | a.load_off[r]];
        }
    }
    double2 th[1 + RB];
    if (has_diag) {
        const double2 *dt = reinterpret_cast<const double2 *>(a.dtab);
#pragma unroll
        for (int v = 0; v <= RB; ++v) th[v] = dt[(size_t)tid * (1 + RB) + v];
        if (tid < (uint32_t)E) q[tid] = dt[((size_t)1 << (T - RB)) * (1 + RB) + tid];
        double2 f = make_double2(1.0, 0.0);
        if (a.d.axis < 3 && tid <= (uint32_t)T) f = reinterpret_cast<const double2 *>(a.wgf)[tile * (T + 1) + tid];
        put_wgf<T>(wgf, a.d, f);
        lds_barrier();
    }
    int cur = a.load_win;
    for (int s = 0; s < a.n_stages; ++s) {
        const uint64_t word = s < kStagesPerWord ? a.st_code[0] : a.st_code[1];
        const uint32_t code = (uint32_t)(word >> (9 * (s % kStagesPerWord))) & 0x1FFu;
        const int w = (int)(code & 15u);
        if (w != cur) {
            any_transpose<RB>(x, lds, cur, w);
            any_transpose<RB>(y, lds, cur, w);
            cur = w;
        }
        if (!((code >> 4) & 1u)) {
            reg_bfly<RB>(x, code >> 5);
            reg_bfly<RB>(y, code >> 5);
        } else {
            reg_diag_pair<T, RB>(x, y, a.d, wgf, th, q, thread_part<RB>(tid, w), base, w);
            if (a.d.axis >= 0 && a.d.axis < 3 && g.np > 0)
                pair_grad<T, RB>(x, y, g, base, w, reinterpret_cast<double *>(lds), red);
        }
    }
    if (cur != a.store_win) {
        any_transpose<RB>(x, lds, cur, a.store_win);
        any_transpose<RB>(y, lds, cur, a.store_win);
    }
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a.store_win), a.tile_runs, a.n_tile_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            psi[gb | a.store_off[r]] = x[r];
            lam[gb | a.store_off[r]] = y[r];
        }
    }
}

// LDS: the transpose buffer (real and imaginary parts in turn for complex128), at least the
// gradient pass's [waves][16][65] doubles.
template <typename R, int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void sweep_pair_kernel(typename Vec<R>::T *__restrict__ psi,
                                                                   typename Vec<R>::T *__restrict__ lam,
                                                                   RegSweepArgs a, PairGradArgs g)
{
    constexpr int NE = 1 << T;
    constexpr int NW = (1 << (T - RB)) / 64 > 0 ? (1 << (T - RB)) / 64 : 1;
    constexpr int NBUF = NE + NE / 16 > NW * 16 * 65 ? NE + NE / 16 : NW * 16 * 65;
    using L = typename std::conditional<sizeof(R) == 8, double, float2>::type;
    __shared__ L lds[NBUF];
    __shared__ double2 wgf[T + 1];
    __shared__ double2 q[1 << RB];
    __shared__ double red[NW * 64];
    reg_sweep_pair<R, T, RB>(psi, lam, a, g, lds, wgf, q, red);
}

// complex128 with half the LDS per workgroup and a register budget for three waves per SIMD:
// three workgroups per CU instead of two at T = 12.
template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(3)))
void sweep_half_kernel(double2 *__restrict__ psi, RegSweepArgs a)
{
    constexpr int NE = 1 << T;
    __shared__ double lds[NE + NE / 16];
    reg_sweep<double, T, RB>(psi, a, lds);
}

// Butterflies of the light-cone stage loop, written in place: (u, v) -> (u + v, (u + v) - 2v).
// A fresh register for u - v would have to be copied back at the end of every masked bit
// (the loop carries the register array): 16 moves per 32 adds.  The difference then carries
// up to one more rounding of the sum (unbiased, like the first), far inside the FP64 error
// budget; for complex64 the 1000-step C(t) error against complex128 stays at the level of
// the exact form (2e-9 at N = 24, GPU test bound 1e-5).
template <typename V>
__device__ __forceinline__ void bfly_inplace(V &a, V &b);
template <>
__device__ __forceinline__ void bfly_inplace(double2 &a, double2 &b)
{
    a.x += b.x;
    a.y += b.y;
    b.x = __builtin_fma(-2.0, b.x, a.x);
    b.y = __builtin_fma(-2.0, b.y, a.y);
}
template <>
__device__ __forceinline__ void bfly_inplace(float2 &a, float2 &b)
{
    a.x += b.x;
    a.y += b.y;
    b.x = __builtin_fmaf(-2.0f, b.x, a.x);
    b.y = __builtin_fmaf(-2.0f, b.y, a.y);
}

template <int RB, typename V>
__device__ __forceinline__ void cone_bfly(V (&x)[1 << RB], uint32_t mask)
{
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        if (!((mask >> v) & 1u)) continue;
#pragma unroll
        for (int r = 0; r < (1 << RB); ++r)
            if (!(r & (1 << v))) bfly_inplace(x[r], x[r | (1 << v)]);
    }
}

// Light-cone transposes.  For disjoint bit fields lds_pos(a | b) = lds_pos(a) + lds_pos(b)
// (no carry out of the low four bits), so an element's LDS slot is the thread's base plus a
// per-register offset that is uniform (scalar) for the window.  The light-cone windows start
// at bit 0 or at a bit >= 4, where lds_pos(r << w) = r * lds_pos(1 << w): the offsets are
// multiples of one scalar stride (forming each from lds_pos took ~8 scalar instructions).  One code path for every pair
// of windows: the stage loop then keeps the register array in place (separate compiled
// variants per window pair made the compiler copy it between registers at every stage).
template <int RB, typename V>
__device__ __forceinline__ void cone_transpose(V (&x)[1 << RB], V *lds, int from, int to)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t bf = lds_pos(thread_part<RB>(tid, from)), bt = lds_pos(thread_part<RB>(tid, to));
    const uint32_t mf = lds_pos(1u << from), mt = lds_pos(1u << to);
    V *pf = lds + bf, *pt = lds + bt;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) pf[r * mf] = x[r];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r] = pt[r * mt];
}

// complex128 through the half buffer: real parts, then imaginary parts
template <int RB>
__device__ __forceinline__ void cone_transpose(double2 (&x)[1 << RB], double *lds, int from, int to)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t bf = lds_pos(thread_part<RB>(tid, from)), bt = lds_pos(thread_part<RB>(tid, to));
    const uint32_t mf = lds_pos(1u << from), mt = lds_pos(1u << to);
    double *pf = lds + bf, *pt = lds + bt;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) pf[r * mf] = x[r].x;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r].x = pt[r * mt];
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) pf[r * mf] = x[r].y;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) x[r].y = pt[r * mt];
}

// Both vectors of the adjoint pair through two buffers at once: half the barriers of two
// transposes in turn.
template <int RB>
__device__ __forceinline__ void cone_transpose_pair(double2 (&x)[1 << RB], double2 (&y)[1 << RB], double *lx,
                                                    double *ly, int from, int to)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t bf = lds_pos(thread_part<RB>(tid, from)), bt = lds_pos(thread_part<RB>(tid, to));
    const uint32_t mf = lds_pos(1u << from), mt = lds_pos(1u << to);
    double *fx = lx + bf, *tx = lx + bt, *fy = ly + bf, *ty = ly + bt;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        fx[r * mf] = x[r].x;
        fy[r * mf] = y[r].x;
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        x[r].x = tx[r * mt];
        y[r].x = ty[r * mt];
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        fx[r * mf] = x[r].y;
        fy[r * mf] = y[r].y;
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        x[r].y = tx[r * mt];
        y[r].y = ty[r * mt];
    }
}
template <int RB, typename V>
__device__ __forceinline__ void cone_transpose_pair(V (&x)[1 << RB], V (&y)[1 << RB], V *lx, V *ly, int from,
                                                    int to)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t bf = lds_pos(thread_part<RB>(tid, from)), bt = lds_pos(thread_part<RB>(tid, to));
    const uint32_t mf = lds_pos(1u << from), mt = lds_pos(1u << to);
    V *fx = lx + bf, *tx = lx + bt, *fy = ly + bf, *ty = ly + bt;
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        fx[r * mf] = x[r];
        fy[r * mf] = y[r];
    }
    lds_barrier();
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        x[r] = tx[r * mt];
        y[r] = ty[r * mt];
    }
}

template <typename V>
__device__ __forceinline__ void apply_cone(V &x, double2 z) { apply_phase(x, z); }

// Row of a phase step's workgroup table that this tile selects (its outside spins).
__device__ __forceinline__ uint64_t cone_row(const ConePhaseArgs &ph, uint64_t tile)
{
    const uint32_t *rb = reinterpret_cast<const uint32_t *>(ph.row_bit);
    uint64_t row = 0;
    for (int b = 0; b < ph.n_row_bits; ++b)
        row |= ((tile >> ((rb[b >> 2] >> (8 * (b & 3))) & 0xffu)) & 1ull) << b;
    return row;
}

// Phase step of a light-cone sweep in window w.  Each step holds few terms, so the product is
// built only from its non-trivial parts: the thread table entry and the workgroup row entry
// (which already hold the couplings and row fields of the window bits with every window bit
// down), the row-dependent fields of the thread bits in xmask, the Gray-code walk over the
// window bits (flipping bit v up multiplies by the square of its two factors); then one
// window-table factor per register.  The walk always runs: a step without such couplings
// has walk factors of exactly 1 + 0i (its tables hold exp(0) there), whose products are
// exact, and a branch on it becomes selects on every register of the walk.  wgf is the
// workgroup's row of the step (w0: its entry 0 times the step's scalar), q the window table.
template <int T, int RB, typename V>
__device__ __forceinline__ void cone_diag(V (&x)[1 << RB], ctab wgf, double2 w0, ctab q,
                                          const double2 (&th)[1 + RB], uint32_t xmask, int w)
{
    const uint32_t tid = threadIdx.x;
    const uint32_t t0 = thread_part<RB>(tid, w);
    double2 p = cmul(w0, th[0]);
    uint32_t m = xmask & ~(((1u << RB) - 1u) << w);
    while (m) {
        const int k = __builtin_ctz(m);
        m &= m - 1u;
        const double2 G = ld2(wgf, 1 + k);
        p = cmul(p, ((t0 >> k) & 1) ? G : make_double2(G.x, -G.y));
    }
    double2 wv[RB];
#pragma unroll
    for (int v = 0; v < RB; ++v) wv[v] = cmul(ld2(wgf, 1 + w + v), th[1 + v]);
#pragma unroll
    for (int k = 0; k < (1 << RB); ++k) {
        const int j = k ^ (k >> 1);
        if (k > 0) {
            const int v = __builtin_ctz(k);
            p = cmul(p, ((j >> v) & 1) ? wv[v] : make_double2(wv[v].x, -wv[v].y));
        }
        apply_cone(x[j], cmul(p, ld2(q, j)));
    }
}

// The same phase step when only the window bits in CM (known when compiling) have walk
// factors other than exactly 1 + 0i: instead of the Gray-code walk over all 2^RB registers,
// the products P[s] = p * prod_{v in s} wv[v] over the subsets s of CM (2^|CM| - 1 complex
// products), and register j takes P[j & CM] * q[j].  Most light-cone steps of a chain couple
// one or two window bits to the rest of the tile (bonds at the window's edges).
template <int T, int RB, uint32_t CM, typename V>
__device__ __forceinline__ void cone_diag_cm(V (&x)[1 << RB], ctab wgf, double2 w0, ctab q,
                                             const double2 (&th)[1 + RB], uint32_t xmask, int w)
{
    const uint32_t t0 = thread_part<RB>(threadIdx.x, w);
    double2 P[1 << RB];
    P[0] = cmul(w0, th[0]);
    uint32_t m = xmask & ~(((1u << RB) - 1u) << w);
    while (m) {
        const int k = __builtin_ctz(m);
        m &= m - 1u;
        const double2 G = ld2(wgf, 1 + k);
        P[0] = cmul(P[0], ((t0 >> k) & 1) ? G : make_double2(G.x, -G.y));
    }
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        if (!((CM >> v) & 1u)) continue;
        const double2 f = cmul(ld2(wgf, 1 + w + v), th[1 + v]);
        const uint32_t lower = CM & ((1u << v) - 1u);
#pragma unroll
        for (uint32_t s = 0; s < (1u << RB); ++s)
            if ((s & ~lower) == 0) P[s | (1u << v)] = cmul(P[s], f);
    }
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) apply_cone(x[j], cmul(P[j & CM], ld2(q, j)));
}

// ... on two vectors (the adjoint's psi and lambda), each factor formed once.  Its own copy
// of the products: sharing them with the one-vector form through a helper made the compiler
// keep part of that form's register array in scratch memory.
template <int T, int RB, uint32_t CM, typename V>
__device__ __forceinline__ void cone_diag_cm_pair(V (&x)[1 << RB], V (&y)[1 << RB], const double2 *wgf,
                                                  const double2 *q, const double2 (&th)[1 + RB],
                                                  uint32_t xmask, int w)
{
    const uint32_t t0 = thread_part<RB>(threadIdx.x, w);
    double2 P[1 << RB];
    P[0] = cmul(wgf[0], th[0]);
    uint32_t m = xmask & ~(((1u << RB) - 1u) << w);
    while (m) {
        const int k = __builtin_ctz(m);
        m &= m - 1u;
        const double2 G = wgf[1 + k];
        P[0] = cmul(P[0], ((t0 >> k) & 1) ? G : make_double2(G.x, -G.y));
    }
#pragma unroll
    for (int v = 0; v < RB; ++v) {
        if (!((CM >> v) & 1u)) continue;
        const double2 f = cmul(wgf[1 + w + v], th[1 + v]);
        const uint32_t lower = CM & ((1u << v) - 1u);
#pragma unroll
        for (uint32_t s = 0; s < (1u << RB); ++s)
            if ((s & ~lower) == 0) P[s | (1u << v)] = cmul(P[s], f);
    }
#pragma unroll
    for (int j = 0; j < (1 << RB); ++j) {
        const double2 z = cmul(P[j & CM], q[j]);
        apply_cone(x[j], z);
        apply_cone(y[j], z);
    }
}

// One phase step of the adjoint light-cone sweep on psi and lambda: the specialised walk
// masks, else subset products over all four bits (the Gray-code walk on two vectors does
// not fit the registers).
template <int T, int RB, typename V>
__device__ __forceinline__ void cone_phase_pair(V (&x)[1 << RB], V (&y)[1 << RB], const ConePhaseArgs &ph,
                                                const double2 *wp, const double2 *qp,
                                                const double2 (&th)[1 + RB], int w)
{
    switch (ph.cmask) {
    case 0: cone_diag_cm_pair<T, RB, 0u>(x, y, wp, qp, th, ph.xmask, w); break;
    case 1: cone_diag_cm_pair<T, RB, 1u>(x, y, wp, qp, th, ph.xmask, w); break;
    case 8: cone_diag_cm_pair<T, RB, 8u>(x, y, wp, qp, th, ph.xmask, w); break;
    case 9: cone_diag_cm_pair<T, RB, 9u>(x, y, wp, qp, th, ph.xmask, w); break;
    default: cone_diag_cm_pair<T, RB, 15u>(x, y, wp, qp, th, ph.xmask, w); break;
    }
}

// The phase tables are reached through pointers stored in the sweep arguments; these name
// global memory, which lets the compiler use global (not flat) loads for them.
typedef const __attribute__((address_space(1))) double *gtab;
__device__ __forceinline__ gtab as_global(const double *p)
{
    return (gtab)(const __attribute__((address_space(1))) void *)p;
}
// a 64-bit value that is the same in every lane, held in scalar registers
__device__ __forceinline__ uint64_t uniform64(uint64_t v)
{
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
}
// complex entry i of a global table of (re, im) pairs
__device__ __forceinline__ double2 gload2(gtab t, size_t i)
{
    return make_double2(t[2 * i], t[2 * i + 1]);
}

__device__ __forceinline__ double wave_sum(double v);

// Observables of a recorded segment from the tile the last light-cone sweep of a vector is
// about to store (its addresses gb | off[r] are the basis indices): FP64 sums over the
// thread's amplitudes, register by register (one bra amplitude in flight at a time keeps the
// register budget of the sweep), then a wave reduction and one row of partials per
// workgroup.  At most kConeRecMax observables per vector.
template <typename R, int RB>
__device__ __forceinline__ void cone_record(const typename Vec<R>::T (&x)[1 << RB], uint64_t gb,
                                            const uint64_t *off, const ConeRec &rec, double *red)
{
    using V = typename Vec<R>::T;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    double acc[kConeRecMax][2];
#pragma unroll
    for (int o = 0; o < kConeRecMax; ++o) acc[o][0] = acc[o][1] = 0.0;
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        const uint64_t b = gb | off[r];
        const double cr = x[r].x, ci = x[r].y, p = cr * cr + ci * ci;
#pragma unroll
        for (int o = 0; o < kConeRecMax; ++o) {
            if (o >= rec.n_obs) break;
            const ObsDev ob = rec.obs[o];
            switch (ob.kind) {
            case 0: acc[o][0] += p; break;
            case 3: acc[o][0] += (((b >> ob.i) & 1) ? 0.5 : -0.5) * p; break;
            case 4: acc[o][0] += ((((b >> ob.i) ^ (b >> ob.j)) & 1) ? -0.25 : 0.25) * p; break;
            case 5: acc[o][0] += ((double)__popcll(b) - 0.5 * rec.n) * p; break;
            case kObsOverlapSz:
            case kObsOverlap: {
                const V w = static_cast<const V *>(rec.bra[o])[b];
                const double s = ob.kind == kObsOverlap ? 1.0 : (((b >> ob.i) & 1) ? 0.5 : -0.5);
                acc[o][0] += s * ((double)w.x * cr + (double)w.y * ci);
                acc[o][1] += s * ((double)w.x * ci - (double)w.y * cr);
                break;
            }
            default: break;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < kConeRecMax; ++o) {
        if (o >= rec.n_obs) break;
        const double a0 = wave_sum(acc[o][0]), a1 = wave_sum(acc[o][1]);
        if (lane == 0) {
            red[2 * wv] = a0;
            red[2 * wv + 1] = a1;
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            double sum = 0.0;
            for (int w = 0; w < nw; ++w) sum += red[2 * w + threadIdx.x];
            rec.partials[(size_t)blockIdx.x * (2 * kMaxObs) + 2 * rec.obs[o].slot + threadIdx.x] = sum;
        }
        __syncthreads();
    }
}

// Every phase step's workgroup row (T + 1 entries) and window table (2^RB entries) into LDS
// (the adjoint's pair sweep, which ran 3% slower with the one-vector sweep's scalar loads).
// Wave v takes the steps v, v + NW, ...: a step's arguments are then uniform (scalar loads;
// the row bits are read as whole words, since scalar loads of single bytes do not exist and
// a vector load would wait behind the tile's), lanes 0..T load its row entries and lanes
// T+1..T+2^RB its window entries, and every step's loads are issued before any is written,
// so they go out right behind the tile's own loads instead of one dependent round trip after
// another.  The caller's barrier makes them visible.
template <int T, int RB>
__device__ __forceinline__ void cone_tables(const ConeArgs *__restrict__ a, uint64_t tile, double2 *wgf,
                                            double2 *qt)
{
    constexpr int E = 1 << RB;
    constexpr uint32_t kThr = 1u << (T - RB);
    const uint32_t tid = threadIdx.x;
    const int nph = a->n_phases;
    constexpr int NW = (int)(kThr / 64);
    constexpr int K = (kConePhases + NW - 1) / NW;
    static_assert(NW >= 1 && T + 1 + E <= 64, "one wave holds a step's tables");
    const int wv = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
    const int lane = (int)(tid & 63);
    const bool row_lane = lane <= T, win_lane = lane > T && lane <= T + E;
    double2 f[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int p = wv + k * NW;
        if (p >= nph) break;
        const ConePhaseArgs &ph = a->ph[p];
        const uint32_t *rb = reinterpret_cast<const uint32_t *>(ph.row_bit);
        uint64_t row = 0;
        for (int b = 0; b < ph.n_row_bits; ++b)
            row |= ((tile >> ((rb[b >> 2] >> (8 * (b & 3))) & 0xffu)) & 1ull) << b;
        // one load instruction for both kinds of lanes (two would share the destination
        // registers, and the second would wait for the first), from uniform table pointers
        const uint64_t pw = uniform64((uint64_t)ph.wgf), pd = uniform64((uint64_t)ph.dtab);
        const uint64_t at = row_lane ? pw + 16 * (row * (T + 1) + lane)
                                     : pd + 16 * ((uint64_t)kThr * (1 + RB) + (lane - T - 1));
        if (row_lane || win_lane) f[k] = gload2(as_global(reinterpret_cast<const double *>(at)), 0);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int p = wv + k * NW;
        if (p >= nph) break;
        if (lane == 0) {
            const ConePhaseArgs &ph = a->ph[p];
            wgf[p * (T + 1)] = cmul(make_double2(ph.kre, ph.kim), f[k]);
        } else if (row_lane) {
            wgf[p * (T + 1) + lane] = f[k];
        } else if (win_lane) {
            qt[p * E + (lane - T - 1)] = f[k];
        }
    }
}

// The thread's row of a phase step's thread table: entry 0 always, entry 1 + v only where
// the step's walk factor for window bit v is not exactly 1 (the stage code lists them).
template <int RB>
__device__ __forceinline__ void cone_thread_row(const ConeArgs *__restrict__ a, uint32_t code, double2 (&th)[1 + RB])
{
    const gtab dt = as_global(a->ph[(code >> 9) & 63u].dtab);
    const uint32_t need = (code >> 15) & 15u;
    // the row offset is formed here, per stage: held across the stage loop it is one register
    // more than the complex128 kernel has, and the compiler spills it
    uint32_t row = threadIdx.x;
    asm volatile("" : "+v"(row));
    th[0] = gload2(dt, (size_t)row * (1 + RB));
#pragma unroll
    for (int v = 0; v < RB; ++v)
        if ((need >> v) & 1u) th[1 + v] = gload2(dt, (size_t)row * (1 + RB) + 1 + v);
}

// Reads one word of every 64-byte line of every phase step's workgroup row and window table,
// right behind the tile's loads: the steps' own scalar loads then hit the scalar cache.  (A
// launch of few workgroups per CU has too few waves to hide a trip to L2 at every step.)
// Wave v takes the steps v, v + NW, ...; every load is issued before any result is used.
template <int T, int RB>
__device__ __forceinline__ void cone_warm(const ConeArgs *__restrict__ a, uint64_t tile)
{
    constexpr int NW = (1 << (T - RB)) / 64;
    constexpr int K = (kConePhases + NW - 1) / NW;
    constexpr int RL = ((T + 1) * 16 + 63) / 64 + 1;   // lines a row can touch
    constexpr int QL = (16 << RB) / 64;                // lines of a window table
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nph = a->n_phases;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int p = wv + k * NW;
        if (p >= nph) break;
        const ConePhaseArgs &ph = a->ph[p];
        acc ^= ctab_touch<RL>(as_const(ph.wgf) + 2 * cone_row(ph, tile) * (T + 1), 16 * (T + 1)) ^
               ctab_touch<QL>(as_const(ph.dtab) + 2 * (1u << (T - RB)) * (1 + RB), 16 << RB);
    }
    asm volatile("" ::"s"(acc));
}

// Light-cone sweep.  The same register windows, transposes and phase arithmetic as the
// register-window sweep, with many phase steps per pass (each restricted to the terms that
// the host assigned to it, with its own workgroup row and tables) and separate tile-bit maps
// for the load and the store.  L is the LDS element of the transposes (double: the half
// buffer for complex128).  The workgroup row and the window table of a phase step are the
// same for every lane: the step reads them with scalar loads where it uses them.
template <typename R, int T, int RB, typename L, bool REC = false>
__device__ __forceinline__ void cone_sweep(typename Vec<R>::T *__restrict__ psi,
                                           const ConeArgs *__restrict__ a, uint64_t tile, L *lds,
                                           const ConeRec *rec = nullptr, double *red = nullptr)
{
    using V = typename Vec<R>::T;
    constexpr int E = 1 << RB;
    const uint32_t tid = threadIdx.x;
    const uint64_t base = dep(tile, a->out_runs, a->n_out_runs);
    V x[E];
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a->load_win), a->load_runs, a->n_load_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) x[r] = ntload(&psi[gb | a->load_off[r]]);
    }
    cone_warm<T, RB>(a, tile);
    // the tile is complete (s_waitcnt vmcnt(0)): the first stage needs it anyway, and the
    // stage loop's waits then cover only the loads it issues itself
    __builtin_amdgcn_s_waitcnt(0x0F70);
    int cur = a->load_win;
    const int ns = a->n_stages;
    for (int s = 0; s < ns; ++s) {
        const uint32_t code = a->st[s];
        const int w = (int)(code & 15u);
        const bool has_phase = (code >> 4) & 1u;
        const int p = (int)((code >> 9) & 63u);
        // the thread's phase-table row is loaded first: its latency then hides behind the
        // transpose and the butterflies of the stage
        double2 th[1 + RB];
        if (has_phase) cone_thread_row<RB>(a, code, th);
        if (w != cur) {
            cone_transpose<RB>(x, lds, cur, w);
            cur = w;
        }
        // butterflies, then (if any) the phase step, in one stage: fewer trips through the
        // stage loop, each of which the compiler ends with copies of the register array
        const uint32_t mask = (code >> 5) & 15u;
        if (mask) cone_bfly<RB>(x, mask);
        if (has_phase) {
            const ConePhaseArgs &ph = a->ph[p];
            const ctab wp = as_const(ph.wgf) + 2 * cone_row(ph, tile) * (T + 1);
            const double2 w0 = cmul(make_double2(ph.kre, ph.kim), ld2(wp, 0));
            const ctab qp = as_const(ph.dtab) + 2 * (1u << (T - RB)) * (1 + RB);
            switch (ph.cmask) {
            case 0: cone_diag_cm<T, RB, 0u>(x, wp, w0, qp, th, ph.xmask, w); break;
            case 1: cone_diag_cm<T, RB, 1u>(x, wp, w0, qp, th, ph.xmask, w); break;
            case 8: cone_diag_cm<T, RB, 8u>(x, wp, w0, qp, th, ph.xmask, w); break;
            case 9: cone_diag_cm<T, RB, 9u>(x, wp, w0, qp, th, ph.xmask, w); break;
            default: cone_diag<T, RB>(x, wp, w0, qp, th, ph.xmask, w); break;
            }
        }
    }
    if (cur != a->store_win) cone_transpose<RB>(x, lds, cur, a->store_win);
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a->store_win), a->store_runs, a->n_store_runs);
        if constexpr (REC) cone_record<R, RB>(x, gb, a->store_off, *rec, red);
#pragma unroll
        for (int r = 0; r < E; ++r) ntstore(&psi[gb | a->store_off[r]], x[r]);
    }
}

// The adjoint's pair sweep stages the phase tables of a sweep (per phase step: T + 1
// workgroup-row entries, then 2^RB window entries) in dynamic LDS sized by the launch for the
// sweep's own phase steps.
template <int T, int RB>
__host__ __device__ constexpr size_t cone_tab_bytes(int n_phases)
{
    return (size_t)n_phases * ((T + 1) + (1 << RB)) * sizeof(double2);
}

// complex128 transposes through the half buffer; three waves per SIMD (at 128 registers,
// which four would need, the compiler spills).  complex64 runs four workgroups per CU.
template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(3)))
void cone_c128_kernel(double2 *__restrict__ psi, const ConeArgs *__restrict__ a, uint64_t n_tiles,
                      int reverse)
{
    constexpr int NE = 1 << T;
    __shared__ double lds[NE + NE / 16];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    cone_sweep<double, T, RB>(psi, a, tile, lds);
}

template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(4)))
void cone_c64_kernel(float2 *__restrict__ psi, const ConeArgs *__restrict__ a, uint64_t n_tiles,
                     int reverse)
{
    constexpr int NE = 1 << T;
    __shared__ float2 lds[NE + NE / 16];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    cone_sweep<float, T, RB>(psi, a, tile, lds);
}

// The last sweep of a vector's recorded segment, with the segment's observables.
template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(3)))
void cone_rec_c128_kernel(double2 *__restrict__ psi, const ConeArgs *__restrict__ a, uint64_t n_tiles,
                          int reverse, ConeRec rec)
{
    constexpr int NE = 1 << T;
    __shared__ double lds[NE + NE / 16];
    __shared__ double red[2 << (T - RB - 6)];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    cone_sweep<double, T, RB, double, true>(psi, a, tile, lds, &rec, red);
}

template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(4)))
void cone_rec_c64_kernel(float2 *__restrict__ psi, const ConeArgs *__restrict__ a, uint64_t n_tiles,
                         int reverse, ConeRec rec)
{
    constexpr int NE = 1 << T;
    __shared__ float2 lds[NE + NE / 16];
    __shared__ double red[2 << (T - RB - 6)];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    cone_sweep<float, T, RB, float2, true>(psi, a, tile, lds, &rec, red);
}

// ------------------------------------------------------------ adjoint light-cone sweep
//
// psi (x) and lambda (y) through one stage program in the same workgroup.  Each phase step
// forms its factors once and applies them to both, then takes the gradient sums of its own
// terms (the fields and bonds of the level that the step applies): per thread the Walsh
// sums M[m] of w_j = Im(conj(y_j) x_j) over the subsets m of the register window (spin
// values +-1/2), and for each term whose window spins form m, M[m] times the spin values of
// its other spins (bits of the thread's index, or of the workgroup's tile index) times the
// step's coefficient, added to the term's accumulator acc[slot][lane] in LDS.  At the end of
// the sweep one thread per accumulator sums its 64 lanes into the workgroup's gradient row.

template <int T, int RB, typename V>
__device__ __forceinline__ void cone_pair_grad(const V (&x)[1 << RB], const V (&y)[1 << RB], double coef,
                                               uint32_t sv, uint32_t tv0, uint32_t tv1, uint32_t t0,
                                               uint32_t tile, double *acc)
{
    constexpr int E = 1 << RB;
    const uint32_t lane = threadIdx.x & 63u;
    double M[E];
#pragma unroll
    for (int j = 0; j < E; ++j) M[j] = (double)y[j].x * (double)x[j].y - (double)y[j].y * (double)x[j].x;
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
        for (int j = 0; j < E; ++j)
            if (!(j & (1 << k))) {
                const double w0 = M[j], w1 = M[j | (1 << k)];
                M[j] = w0 + w1;
                M[j | (1 << k)] = 0.5 * (w1 - w0);
            }
    // a spin that is down contributes -1/2, one that is up +1/2: the sign is the parity of the
    // term's masked bits that are 0, set directly in the sign bit
    const uint32_t nt0 = ~t0, ntile = ~tile;
    auto term = [&](double base, int t) {
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane((int)tv0, t);
        const uint32_t w1 = (uint32_t)__builtin_amdgcn_readlane((int)tv1, t);
        const uint32_t par = __popc((w0 >> 12) & nt0) + __popc(w1 & ntile);
        const double v = __builtin_ldexp(base, -(int)((w0 >> 8) & 3u));
        atomicAdd(&acc[(w0 & 0xffu) * 64 + lane],
                  __hiloint2double(__double2hiint(v) ^ (int)(par << 31), __double2loint(v)));
    };
#pragma unroll
    for (int m = 0; m < E; ++m) {
        const int t1 = __builtin_amdgcn_readlane((int)sv, m + 1);
        const double base = coef * M[m];
        for (int t = __builtin_amdgcn_readlane((int)sv, m); t < t1; ++t) term(base, t);
    }
}

template <typename R, int T, int RB, typename L>
__device__ __forceinline__ void cone_pair_sweep(typename Vec<R>::T *__restrict__ psi,
                                                typename Vec<R>::T *__restrict__ lam,
                                                const ConeArgs *__restrict__ a,
                                                const ConeGradArgs *__restrict__ g, double *slots,
                                                int stride, uint64_t tile, L *lds, double2 *wgf,
                                                double2 *qt, double *acc)
{
    using V = typename Vec<R>::T;
    constexpr int E = 1 << RB;
    constexpr uint32_t kThr = 1u << (T - RB);
    constexpr int HB = (1 << T) + (1 << T) / 16;   // one transpose buffer; lds holds two
    const uint32_t tid = threadIdx.x;
    const uint64_t base = dep(tile, a->out_runs, a->n_out_runs);
    V x[E], y[E];
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a->load_win), a->load_runs, a->n_load_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            x[r] = ntload(&psi[gb | a->load_off[r]]);
            y[r] = ntload(&lam[gb | a->load_off[r]]);
        }
    }
    cone_tables<T, RB>(a, tile, wgf, qt);
    const int n_slots = g->n_slots;
    for (int i = (int)tid; i < n_slots * 64; i += (int)kThr) acc[i] = 0.0;
    lds_barrier();
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): as in cone_sweep
    int cur = a->load_win;
    const int ns = a->n_stages;
    for (int s = 0; s < ns; ++s) {
        const uint32_t code = a->st[s];
        const int w = (int)(code & 15u);
        const bool has_phase = (code >> 4) & 1u;
        const int p = (int)((code >> 9) & 63u);
        double2 th[1 + RB];
        uint32_t sv = 0, tv0 = 0, tv1 = 0;   // the step's term offsets and terms, one per lane
        if (has_phase) {
            cone_thread_row<RB>(a, code, th);
            const uint32_t lane = tid & 63u;
            sv = (uint32_t)g->start[p][lane & 31u];
            tv0 = g->term[p][0][lane];
            tv1 = g->term[p][1][lane];
        }
        if (w != cur) {
            cone_transpose_pair<RB>(x, y, lds, lds + HB, cur, w);
            cur = w;
        }
        const uint32_t mask = (code >> 5) & 15u;
        if (mask) {
            cone_bfly<RB>(x, mask);
            cone_bfly<RB>(y, mask);
        }
        if (has_phase) {
            cone_phase_pair<T, RB>(x, y, a->ph[p], wgf + p * (T + 1), qt + p * E, th, w);
            cone_pair_grad<T, RB>(x, y, g->coef[p], sv, tv0, tv1, thread_part<RB>(tid, w), (uint32_t)tile, acc);
        }
    }
    if (cur != a->store_win) cone_transpose_pair<RB>(x, y, lds, lds + HB, cur, a->store_win);
    {
        const uint64_t gb = base | dep(thread_part<RB>(tid, a->store_win), a->store_runs, a->n_store_runs);
#pragma unroll
        for (int r = 0; r < E; ++r) {
            ntstore(&psi[gb | a->store_off[r]], x[r]);
            ntstore(&lam[gb | a->store_off[r]], y[r]);
        }
    }
    __syncthreads();
    for (int i = (int)tid; i < n_slots; i += (int)kThr) {
        double sum = 0.0;
        for (int l = 0; l < 64; ++l) sum += acc[i * 64 + l];
        slots[(size_t)blockIdx.x * stride + g->col[i]] += sum;
    }
}

// Static LDS: a transpose buffer per vector; dynamic LDS: the phase tables (cone_tab_bytes),
// then the accumulators.
template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void cone_pair_c128_kernel(double2 *__restrict__ psi,
                                                                       double2 *__restrict__ lam,
                                                                       const ConeArgs *__restrict__ a,
                                                                       const ConeGradArgs *__restrict__ g,
                                                                       double *slots, int stride,
                                                                       uint64_t n_tiles, int reverse)
{
    constexpr int NE = 1 << T;
    __shared__ double lds[2 * (NE + NE / 16)];
    extern __shared__ double2 cone_dyn[];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    const int nph = a->n_phases;
    double2 *qt = cone_dyn + nph * (T + 1);
    cone_pair_sweep<double, T, RB>(psi, lam, a, g, slots, stride, tile, lds, cone_dyn, qt,
                                   reinterpret_cast<double *>(qt + (nph << RB)));
}

template <int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void cone_pair_c64_kernel(float2 *__restrict__ psi,
                                                                      float2 *__restrict__ lam,
                                                                      const ConeArgs *__restrict__ a,
                                                                      const ConeGradArgs *__restrict__ g,
                                                                      double *slots, int stride,
                                                                      uint64_t n_tiles, int reverse)
{
    constexpr int NE = 1 << T;
    __shared__ float2 lds[2 * (NE + NE / 16)];
    extern __shared__ double2 cone_dyn[];
    const uint64_t tile = reverse ? n_tiles - 1 - blockIdx.x : blockIdx.x;
    const int nph = a->n_phases;
    double2 *qt = cone_dyn + nph * (T + 1);
    cone_pair_sweep<float, T, RB>(psi, lam, a, g, slots, stride, tile, lds, cone_dyn, qt,
                                  reinterpret_cast<double *>(qt + (nph << RB)));
}

// Batched: workgroup b works on tile b % tiles_per_chain of chain c = b / tiles_per_chain: its
// state starts at element off[c] of the packed buffer and its arguments for this sweep are
// args[c].  (Both are derived from kernel arguments, so the stage loop keeps its scalar
// loads and the state accesses stay global ones; pointers read from memory lose both.)
template <typename R, int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) __attribute__((amdgpu_waves_per_eu(3)))
void cone_batch_kernel(typename Vec<R>::T *__restrict__ packed, const int64_t *__restrict__ off,
                       const ConeArgs *__restrict__ args, uint64_t tiles_per_chain, int reverse)
{
    constexpr int NE = 1 << T;
    using L = typename std::conditional<sizeof(R) == 8, double, float2>::type;
    __shared__ L lds[NE + NE / 16];
    const uint64_t c = blockIdx.x / tiles_per_chain;
    uint64_t tile = blockIdx.x - c * tiles_per_chain;
    if (reverse) tile = tiles_per_chain - 1 - tile;
    cone_sweep<R, T, RB>(packed + off[c], args + c, tile, lds);
}

// Marks registers as produced here: the compiler then waits for their loads once, at this
// point, instead of conservatively inside the stage loop (where it would also wait for the
// next tile's prefetch).  Each amplitude passes through the empty asm as one whole vector
// register tuple (splitting it into its two halves as separate operands miscompiles the
// complex128 case: the store address was allocated over the imaginary half).
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <int RB>
__device__ __forceinline__ void settle(double2 (&x)[1 << RB])
{
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        u32x4_t t = __builtin_bit_cast(u32x4_t, x[r]);
        asm volatile("" : "+v"(t));
        x[r] = __builtin_bit_cast(double2, t);
    }
}
template <int RB>
__device__ __forceinline__ void settle(float2 (&x)[1 << RB])
{
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) {
        u32x2_t t = __builtin_bit_cast(u32x2_t, x[r]);
        asm volatile("" : "+v"(t));
        x[r] = __builtin_bit_cast(float2, t);
    }
}

// Stages and store of one tile held in registers (shared by the pipelined sweep).
template <int T, int RB, typename V>
__device__ __forceinline__ void pipe_tile(V (&x)[1 << RB], V *__restrict__ psi, const RegSweepArgs &a,
                                          V *lds, double2 *wgf, const double2 (&th)[1 + RB],
                                          const double2 *q, uint64_t base, uint64_t spart)
{
    const uint32_t tid = threadIdx.x;
    int cur = a.load_win;
    for (int s = 0; s < a.n_stages; ++s) {
        const uint64_t word = s < kStagesPerWord ? a.st_code[0] : a.st_code[1];
        const uint32_t code = (uint32_t)(word >> (9 * (s % kStagesPerWord))) & 0x1FFu;
        const int w = (int)(code & 15u);
        if (w != cur) {
            reg_transpose<RB>(x, lds, cur, w);
            cur = w;
        }
        if (!((code >> 4) & 1u)) {
            reg_bfly<RB>(x, code >> 5);
        } else {
            reg_diag_tab<T, RB>(x, a.d, wgf, wgf[0], th, q, thread_part<RB>(tid, w), base, w);
        }
    }
    if (cur != a.store_win) reg_transpose<RB>(x, lds, cur, a.store_win);
#pragma unroll
    for (int r = 0; r < (1 << RB); ++r) (psi + (base | a.store_off[r]))[spart] = x[r];
}

// Pipelined register-window sweep: a grid of resident workgroups walks the tiles with a
// stride of gridDim.x, alternating two register sets.  The global loads of the next tile
// (and its row of workgroup phase factors) are issued before the current tile's stages
// run, so each workgroup keeps HBM busy while it computes even when the LDS footprint
// allows only one or two workgroups per CU.  Stores are fire-and-forget.  Single state
// only (no batched chains).
template <typename R, int T, int RB>
__global__ __launch_bounds__(1 << (T - RB)) void sweep_pipe_kernel(typename Vec<R>::T *__restrict__ psi,
                                                                   RegSweepArgs a)
{
    using V = typename Vec<R>::T;
    constexpr int E = 1 << RB;
    constexpr int NE = 1 << T;
    __shared__ V lds[NE + NE / 16];
    __shared__ double2 wgf[2][T + 1];   // one per register set: no barrier needed before refilling
    __shared__ double2 q[E];
    const uint32_t tid = threadIdx.x;
    const uint64_t stride = gridDim.x;
    uint64_t tile = blockIdx.x;   // walk index; the tile itself is phys(tile)
    if (tile >= a.n_tiles) return;
    const uint64_t last = a.reverse ? a.n_tiles - 1 : 0;
    auto phys = [&](uint64_t t) { return a.reverse ? last - t : t; };
    const bool has_diag = a.diag_win >= 0;
    // a.wgf is never NULL here (the host passes a one-entry unit row for phase steps without
    // energy), so the loads below need no branch and stay global loads
    const bool has_wg = has_diag && a.d.axis < 3 && tid <= (uint32_t)T;
    const double2 *wgt = reinterpret_cast<const double2 *>(a.wgf);
    // Addresses: the tile base and the register offsets are uniform (scalar); only the
    // thread part is per lane, so no per-register 64-bit addresses stay live in VGPRs.
    const uint64_t lpart = dep(thread_part<RB>(tid, a.load_win), a.tile_runs, a.n_tile_runs);
    const uint64_t spart = dep(thread_part<RB>(tid, a.store_win), a.tile_runs, a.n_tile_runs);
    V xa[E], xb[E];
    double2 fa, fb;
    {
        const uint64_t tb = dep(phys(tile), a.out_runs, a.n_out_runs);
        fa = wgt[has_wg ? phys(tile) * (T + 1) + tid : 0];
#pragma unroll
        for (int r = 0; r < E; ++r) xa[r] = (psi + (tb | a.load_off[r]))[lpart];
    }
    double2 th[1 + RB];
    if (has_diag) {
        const double2 *dt = reinterpret_cast<const double2 *>(a.dtab);
#pragma unroll
        for (int v = 0; v <= RB; ++v) th[v] = dt[(size_t)tid * (1 + RB) + v];
        if (tid < (uint32_t)E) q[tid] = dt[((size_t)1 << (T - RB)) * (1 + RB) + tid];
    }
    // The prefetch is unconditional (past the end it re-reads the current tile and the data
    // is never used): a branch around it would make the compiler wait for it before the
    // stages, where the paths merge.
    for (;;) {
        // set A holds `tile` (loads in flight); prefetch the next tile into set B
        uint64_t next = tile + stride;
        {
            const uint64_t pf = phys(next < a.n_tiles ? next : tile);
            const uint64_t tb = dep(pf, a.out_runs, a.n_out_runs);
            fb = wgt[has_wg ? pf * (T + 1) + tid : 0];
#pragma unroll
            for (int r = 0; r < E; ++r) xb[r] = (psi + (tb | a.load_off[r]))[lpart];
        }
        settle<RB>(xa);
        if (has_diag) {
            put_wgf<T>(wgf[0], a.d, has_wg ? fa : make_double2(1.0, 0.0));
            lds_barrier();
        }
        pipe_tile<T, RB>(xa, psi, a, lds, wgf[0], th, q, dep(phys(tile), a.out_runs, a.n_out_runs), spart);
        tile = next;
        if (tile >= a.n_tiles) break;
        // set B holds `tile`; prefetch the next tile into set A
        next = tile + stride;
        {
            const uint64_t pf = phys(next < a.n_tiles ? next : tile);
            const uint64_t tb = dep(pf, a.out_runs, a.n_out_runs);
            fa = wgt[has_wg ? pf * (T + 1) + tid : 0];
#pragma unroll
            for (int r = 0; r < E; ++r) xa[r] = (psi + (tb | a.load_off[r]))[lpart];
        }
        settle<RB>(xb);
        if (has_diag) {
            put_wgf<T>(wgf[1], a.d, has_wg ? fb : make_double2(1.0, 0.0));
            lds_barrier();
        }
        pipe_tile<T, RB>(xb, psi, a, lds, wgf[1], th, q, dep(phys(tile), a.out_runs, a.n_out_runs), spart);
        tile = next;
        if (tile >= a.n_tiles) break;
    }
}

// Whole-state kernel: one workgroup per vector runs every (phase, layer) pass of a segment.
// For n < 8 the T = 8 instance is used with only 2^n amplitudes live.
__device__ __forceinline__ double wave_sum(double v);

// FP64 observables of the LDS-resident state (real kinds: norm, S^x, S^y, S^z of a spin,
// S^z S^z, M^z), written to out[slot].  Every thread of the workgroup calls it.
template <typename V>
__device__ void resident_record(const V *tile, int ne, int n, const ObsDev *obs, int n_obs,
                                double *out)
{
    __shared__ double red[kThreads / 64][kMaxObs];
    double acc[kMaxObs];
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) acc[o] = 0.0;
    for (int t = threadIdx.x; t < ne; t += kThreads) {
        const V c = tile[t];
        const double cr = c.x, ci = c.y, p = cr * cr + ci * ci;
#pragma unroll
        for (int o = 0; o < kMaxObs; ++o) {
            if (o >= n_obs) continue;
            const ObsDev ob = obs[o];
            switch (ob.kind) {
            case 0: acc[o] += p; break;
            case 3: acc[o] += (((t >> ob.i) & 1) ? 0.5 : -0.5) * p; break;
            case 4: acc[o] += ((((t >> ob.i) ^ (t >> ob.j)) & 1) ? -0.25 : 0.25) * p; break;
            case 5: acc[o] += ((double)__builtin_popcount(t) - 0.5 * n) * p; break;
            case 1:
            case 2:
                if (!((t >> ob.i) & 1)) {
                    const V u = tile[t | (1 << ob.i)];
                    const double zr = cr * u.x + ci * u.y, zi = cr * u.y - ci * u.x;
                    acc[o] += (ob.kind == 1) ? zr : -zi;
                }
                break;
            default: break;
            }
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) {
        if (o >= n_obs) continue;
        const double s = wave_sum(acc[o]);
        if (lane == 0) red[wv][o] = s;
    }
    __syncthreads();
    if (threadIdx.x < n_obs) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        out[obs[threadIdx.x].slot] = s;
    }
    __syncthreads();
}

template <typename R, int T>
__global__ __launch_bounds__(kThreads) void resident_kernel(ResidentArgs a)
{
    using V = typename Vec<R>::T;
    constexpr int NV = T - kFixedBits;
    __shared__ V tile[1 << T];
    __shared__ double2 qtab[1 << NV];
    V *psi;
    const double *wg[3], *jt[3];
    double *rec = nullptr;
    if (a.chains) {  // batched: one chain per workgroup
        const ResidentChain ch = a.chains[blockIdx.x];
        psi = static_cast<V *>(ch.psi);
        for (int x = 0; x < 3; ++x) {
            wg[x] = ch.wg[x];
            jt[x] = ch.jt[x];
        }
        rec = ch.rec;
    } else {
        psi = reinterpret_cast<V *>(a.psi[blockIdx.x]);
        for (int x = 0; x < 3; ++x) {
            wg[x] = a.wg[x];
            jt[x] = a.jt[x];
        }
    }
    const int ne = 1 << a.n;
    for (int t = threadIdx.x; t < ne; t += kThreads) tile[t] = psi[t];
    __syncthreads();
    const uint32_t all = (uint32_t)(ne - 1);
    const int reps = a.n_rep > 0 ? a.n_rep : 1;
    for (int r = 0; r < reps; ++r) {
        for (int s = 0; s < a.n_ops; ++s) {
            const ResidentOp op = a.ops[s];
            if (op.fac) {
                for (int t = threadIdx.x; t < ne; t += kThreads) apply_phase(tile[t], op.fac[t]);
                __syncthreads();
            } else if (op.d.axis >= 0) {
                const int ax = op.d.axis < 3 ? op.d.axis : 0;
                build_qtab<T>(qtab, op.d, jt[ax]);
                __syncthreads();
                diag_step<T>(tile, ne, op.d, wg[ax], jt[ax], qtab, (uint64_t)threadIdx.x);
                __syncthreads();
            }
            if (op.post) wht_layer(tile, ne, all);
            if (op.rec >= 0 && rec) resident_record(tile, ne, a.n, a.obs, a.n_obs, rec + (size_t)op.rec * a.slots);
        }
        if (a.rec_rows) resident_record(tile, ne, a.n, a.obs, a.n_obs, a.rec_rows + (size_t)r * a.slots);
    }
    for (int t = threadIdx.x; t < ne; t += kThreads) psi[t] = tile[t];
}

// Phase factors of the resident ops, one workgroup per op: the op's phase step applied to a
// tile of ones leaves in each entry exactly the factor that the step multiplies that
// amplitude by (the product with 1 + 0i is exact), so applying the stored factors gives
// the same amplitudes as forming them in the resident kernel.
template <int T>
__global__ __launch_bounds__(kThreads) void resident_factor_kernel(ResidentArgs a, double2 *out)
{
    constexpr int NV = T - kFixedBits;
    __shared__ double2 tile[1 << T];
    __shared__ double2 qtab[1 << NV];
    const ResidentOp op = a.ops[blockIdx.x];
    if (op.d.axis < 0) return;
    const int ne = 1 << a.n;
    for (int t = threadIdx.x; t < ne; t += kThreads) tile[t] = make_double2(1.0, 0.0);
    const int ax = op.d.axis < 3 ? op.d.axis : 0;
    build_qtab<T>(qtab, op.d, a.jt[ax]);
    __syncthreads();
    diag_step<T>(tile, ne, op.d, a.wg[ax], a.jt[ax], qtab, (uint64_t)threadIdx.x);
    __syncthreads();
    double2 *o = out + ((size_t)blockIdx.x << a.n);
    for (int t = threadIdx.x; t < ne; t += kThreads) o[t] = tile[t];
}

// ----------------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Share of <psi|H|psi> (H of Sec. 2, Eq. 1) owned by basis index b: the diagonal part
// D_z(b)|c_b|^2, and for every pair of basis states that an x or y term connects, twice
// the real part of its matrix element, counted at the member whose flipped bits are clear.
// S^x flips a spin with amplitude 1/2, S^y with +i/2 from down to up (bit clear to set)
// and -i/2 back, so for one spin q and c = c_b, u = c_{b + 2^q} (bit q of b clear):
//   h^x <S^x_q> + h^y <S^y_q>  gathers  h^x Re(conj(c) u) - h^y Im(conj(c) u),
// and for a bond (i, j) with both bits of b clear, A = Re(conj(c_00) c_11),
// B = Re(conj(c_01) c_10):  J^x <S^x S^x> + J^y <S^y S^y>  gathers  (J^x (A + B) + J^y (B - A)) / 2.
template <typename V>
__device__ __noinline__ double energy_density(const V *__restrict__ ket, uint64_t b, int n,
                                              const double *__restrict__ hf,
                                              const HamBond *__restrict__ hb, int nb)
{
    const V c = ket[b];
    const double cr = c.x, ci = c.y;
    double dz = 0.0, off = 0.0;
    for (int q = 0; q < n; ++q) {
        const bool up = (b >> q) & 1;
        dz += hf[3 * q + 2] * (up ? 0.5 : -0.5);
        const double hx = hf[3 * q], hy = hf[3 * q + 1];
        if (!up && (hx != 0.0 || hy != 0.0)) {
            const V u = ket[b | (1ull << q)];
            const double zr = cr * u.x + ci * u.y, zi = cr * u.y - ci * u.x;
            off += hx * zr - hy * zi;
        }
    }
    for (int k = 0; k < nb; ++k) {
        const HamBond t = hb[k];
        const uint64_t mi = 1ull << t.i, mj = 1ull << t.j;
        dz += t.jz * ((((b >> t.i) ^ (b >> t.j)) & 1) ? -0.25 : 0.25);
        if ((t.jx != 0.0 || t.jy != 0.0) && !(b & (mi | mj))) {
            const V c11 = ket[b | mi | mj], c01 = ket[b | mi], c10 = ket[b | mj];
            const double A = cr * c11.x + ci * c11.y;
            const double B = (double)c01.x * c10.x + (double)c01.y * c10.y;
            off += 0.5 * (t.jx * (A + B) + t.jy * (B - A));
        }
    }
    return dz * (cr * cr + ci * ci) + off;
}

template <typename R>
__global__ __launch_bounds__(kThreads) void reduce_kernel(ReduceArgs a, double *partials)
{
    using V = typename Vec<R>::T;
    double acc[kMaxObs][2];
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) acc[o][0] = acc[o][1] = 0.0;
    const uint64_t dim = 1ull << a.n;
    const uint64_t stride = (uint64_t)gridDim.x * kThreads;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < dim; b += stride) {
#pragma unroll
        for (int o = 0; o < kMaxObs; ++o) {
            if (o >= a.n_obs) continue;
            const ObsDev ob = a.obs[o];
            const V *ket = reinterpret_cast<const V *>(a.psi[ob.ket]);
            const V c = ket[b];
            const double cr = c.x, ci = c.y;
            const double p = cr * cr + ci * ci;
            switch (ob.kind) {
            case 0: acc[o][0] += p; break;
            case 3: acc[o][0] += (((b >> ob.i) & 1) ? 0.5 : -0.5) * p; break;
            case 4:
                acc[o][0] += ((((b >> ob.i) ^ (b >> ob.j)) & 1) ? -0.25 : 0.25) * p;
                break;
            case 5: acc[o][0] += ((double)__popcll(b) - 0.5 * a.n) * p; break;
            case 1:
            case 2:
                if (!((b >> ob.i) & 1)) {
                    const V u = ket[b | (1ull << ob.i)];
                    // conj(c) * u
                    const double zr = cr * u.x + ci * u.y, zi = cr * u.y - ci * u.x;
                    acc[o][0] += (ob.kind == 1) ? zr : -zi;
                }
                break;
            case 6: acc[o][0] += energy_density<V>(ket, b, a.n, a.ham_h, a.ham_b, a.ham_nb); break;
            case kObsSxSx:
            case kObsSySy: {
                // pairs (b, b + 2^i + 2^j) and (b + 2^i, b + 2^j) at the member with both bits clear
                const uint64_t mi = 1ull << ob.i, mj = 1ull << ob.j;
                if (!(b & (mi | mj))) {
                    const V c11 = ket[b | mi | mj], c01 = ket[b | mi], c10 = ket[b | mj];
                    const double A = cr * c11.x + ci * c11.y;
                    const double B = (double)c01.x * c10.x + (double)c01.y * c10.y;
                    acc[o][0] += 0.5 * (ob.kind == kObsSxSx ? A + B : B - A);
                }
                break;
            }
            case kObsOverlap: {
                const V *bra = reinterpret_cast<const V *>(a.psi[ob.bra]);
                const V w = bra[b];
                acc[o][0] += (double)w.x * cr + (double)w.y * ci;
                acc[o][1] += (double)w.x * ci - (double)w.y * cr;
                break;
            }
            case 7: {
                const V *bra = reinterpret_cast<const V *>(a.psi[ob.bra]);
                const V w = bra[b];
                const double s = ((b >> ob.i) & 1) ? 0.5 : -0.5;
                acc[o][0] += s * ((double)w.x * cr + (double)w.y * ci);
                acc[o][1] += s * ((double)w.x * ci - (double)w.y * cr);
                break;
            }
            default: break;
            }
        }
    }
    __shared__ double red[kThreads / 64][kMaxObs * 2];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) {
        if (o >= a.n_obs) continue;
        const double s0 = wave_sum(acc[o][0]), s1 = wave_sum(acc[o][1]);
        if (lane == 0) {
            red[wv][2 * o] = s0;
            red[wv][2 * o + 1] = s1;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * a.n_obs) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        partials[(size_t)blockIdx.x * (2 * kMaxObs) + threadIdx.x] = s;
    }
}

// Sum the per-block partials in a fixed order and write the requested slots: one wavefront
// per slot, each lane a Neumaier-compensated strided sum, then a fixed shuffle tree.
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double *partials, int nblocks,
                                                            ReduceArgs a, double *out)
{
    const int lane = threadIdx.x & 63;
    for (int s = threadIdx.x >> 6; s < 2 * a.n_obs; s += kThreads / 64) {
        double acc = 0.0, comp = 0.0;
        for (int b = lane; b < nblocks; b += 64) {
            const double x = partials[(size_t)b * (2 * kMaxObs) + s];
            const double t = acc + x;
            comp += (fabs(acc) >= fabs(x)) ? (acc - t) + x : (x - t) + acc;
            acc = t;
        }
        const double tot = wave_sum(acc + comp);
        const int o = s >> 1, part = s & 1;
        const ObsDev ob = a.obs[o];
        if (lane == 0 && (part == 0 || obs_complex(ob.kind))) out[ob.slot + part] = tot;
    }
}

// Batched observables: blockIdx.y = chain, the chain's vector split over gridDim.x blocks;
// partials[(chain * gridDim.x + block) * kMaxObs + o].
template <typename R>
__global__ __launch_bounds__(kThreads) void batch_reduce_kernel(BatchReduceArgs a, double *partials)
{
    using V = typename Vec<R>::T;
    const ChainPtrs cp = a.chains[blockIdx.y];
    const V *psi = static_cast<const V *>(cp.psi);
    double acc[kMaxObs];
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) acc[o] = 0.0;
    const uint64_t dim = 1ull << a.n;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kThreads) {
        const V c = psi[b];
        const double cr = c.x, ci = c.y, p = cr * cr + ci * ci;
#pragma unroll
        for (int o = 0; o < kMaxObs; ++o) {
            if (o >= a.n_obs) continue;
            const ObsDev ob = a.obs[o];
            switch (ob.kind) {
            case 0: acc[o] += p; break;
            case 3: acc[o] += (((b >> ob.i) & 1) ? 0.5 : -0.5) * p; break;
            case 4: acc[o] += ((((b >> ob.i) ^ (b >> ob.j)) & 1) ? -0.25 : 0.25) * p; break;
            case 5: acc[o] += ((double)__popcll(b) - 0.5 * a.n) * p; break;
            case 1:
            case 2:
                if (!((b >> ob.i) & 1)) {
                    const V u = psi[b | (1ull << ob.i)];
                    const double zr = cr * u.x + ci * u.y, zi = cr * u.y - ci * u.x;
                    acc[o] += (ob.kind == 1) ? zr : -zi;
                }
                break;
            default: break;
            }
        }
    }
    __shared__ double red[kThreads / 64][kMaxObs];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int o = 0; o < kMaxObs; ++o) {
        if (o >= a.n_obs) continue;
        const double s = wave_sum(acc[o]);
        if (lane == 0) red[wv][o] = s;
    }
    __syncthreads();
    if (threadIdx.x < a.n_obs) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        partials[((size_t)blockIdx.y * gridDim.x + blockIdx.x) * kMaxObs + threadIdx.x] = s;
    }
}

// One workgroup per chain: sum its blocks' partials in order, write record a.rec.
__global__ __launch_bounds__(kThreads) void batch_finalize_kernel(BatchReduceArgs a, const double *partials,
                                                                  int nbpc)
{
    const ChainPtrs cp = a.chains[blockIdx.x];
    const int lane = threadIdx.x & 63;
    for (int o = threadIdx.x >> 6; o < a.n_obs; o += kThreads / 64) {
        double s = 0.0;
        for (int b = lane; b < nbpc; b += 64) s += partials[((size_t)blockIdx.x * nbpc + b) * kMaxObs + o];
        s = wave_sum(s);
        if (lane == 0) cp.rec[(size_t)a.rec * a.slots + a.obs[o].slot] = s;
    }
}

// --------------------------------------------------------------------------- adjoint

// out = O psi for the Hermitian observables (S^x, S^y, S^z of one spin, S^z S^z, M^z).
template <typename R>
__global__ __launch_bounds__(kThreads) void apply_obs_kernel(const typename Vec<R>::T *__restrict__ psi,
                                                             typename Vec<R>::T *__restrict__ out,
                                                             int kind, int i, int j, int n)
{
    using V = typename Vec<R>::T;
    const uint64_t dim = 1ull << n;
    const uint64_t m = 1ull << i;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kThreads) {
        V o;
        if (kind == 1 || kind == 2) {
            const V c = psi[b ^ m];
            if (kind == 1) {  // (S^x psi)_b = c_{b^m} / 2
                o.x = (R)0.5 * c.x;
                o.y = (R)0.5 * c.y;
            } else {          // (S^y psi)_b = (i/2) sigma c_{b^m}, sigma = +1 for a clear bit
                const R sg = ((b >> i) & 1) ? (R)-0.5 : (R)0.5;
                o.x = -sg * c.y;
                o.y = sg * c.x;
            }
        } else {
            double f;
            if (kind == 3) f = ((b >> i) & 1) ? 0.5 : -0.5;
            else if (kind == 4) f = (((b >> i) ^ (b >> j)) & 1) ? -0.25 : 0.25;
            else f = (double)__popcll(b) - 0.5 * n;
            const V c = psi[b];
            o.x = (R)(f * c.x);
            o.y = (R)(f * c.y);
        }
        out[b] = o;
    }
}

// out = H psi, gathered per basis index b (H of Sec. 2, Eq. 1):
//   (H psi)_b = D_z(b) c_b + sum_q (h^x_q / 2 + s_q h^y_q / 2) c_{b ^ 2^q}
//             + sum_bonds (J^x / 4 + t_ij J^y / 4) c_{b ^ 2^i ^ 2^j},
// with s_q = +i if bit q of b is clear and -i if set (S^y takes up to down with +i/2), and
// t_ij = -1 if bits i and j of b are equal, +1 otherwise (the product of two such factors).
template <typename R>
__global__ __launch_bounds__(kThreads) void apply_ham_kernel(const typename Vec<R>::T *__restrict__ psi,
                                                             typename Vec<R>::T *__restrict__ out, int n,
                                                             const double *__restrict__ hf,
                                                             const HamBond *__restrict__ hb, int nb)
{
    using V = typename Vec<R>::T;
    const uint64_t dim = 1ull << n;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kThreads) {
        const V c = psi[b];
        double dz = 0.0, orr = 0.0, oi = 0.0;
        for (int q = 0; q < n; ++q) {
            const bool up = (b >> q) & 1;
            dz += hf[3 * q + 2] * (up ? 0.5 : -0.5);
            const double hx = hf[3 * q], hy = hf[3 * q + 1];
            if (hx != 0.0 || hy != 0.0) {
                const V u = psi[b ^ (1ull << q)];
                const double sy = up ? -0.5 * hy : 0.5 * hy;   // (i sy) u
                orr += 0.5 * hx * u.x - sy * u.y;
                oi += 0.5 * hx * u.y + sy * u.x;
            }
        }
        for (int k = 0; k < nb; ++k) {
            const HamBond t = hb[k];
            const bool eq = !((((b >> t.i) ^ (b >> t.j)) & 1));
            dz += t.jz * (eq ? 0.25 : -0.25);
            if (t.jx != 0.0 || t.jy != 0.0) {
                const V u = psi[b ^ (1ull << t.i) ^ (1ull << t.j)];
                const double w = 0.25 * (t.jx + (eq ? -t.jy : t.jy));
                orr += w * u.x;
                oi += w * u.y;
            }
        }
        V o;
        o.x = (R)(dz * c.x + orr);
        o.y = (R)(dz * c.y + oi);
        out[b] = o;
    }
}

// Per-block partial sums of  sum_b f_p(b) Im(conj(lam_b) psi_b)  for a chunk of parameters
// (f = s_i for a field, s_i s_j for a coupling); both vectors are in the frame of the
// phase step that was applied last.
template <typename R>
__global__ __launch_bounds__(kThreads) void grad_reduce_kernel(const typename Vec<R>::T *__restrict__ psi,
                                                               const typename Vec<R>::T *__restrict__ lam,
                                                               GradArgs a)
{
    using V = typename Vec<R>::T;
    double acc[kGradChunk];
#pragma unroll
    for (int p = 0; p < kGradChunk; ++p) acc[p] = 0.0;
    const uint64_t dim = 1ull << a.n;
    for (uint64_t b = (uint64_t)blockIdx.x * kThreads + threadIdx.x; b < dim;
         b += (uint64_t)gridDim.x * kThreads) {
        const V u = psi[b], l = lam[b];
        const double w = (double)l.x * (double)u.y - (double)l.y * (double)u.x;
#pragma unroll
        for (int p = 0; p < kGradChunk; ++p) {
            if (p >= a.np) continue;
            const int i = a.pi[p], j = a.pj[p];
            double f;
            if (j < 0) f = ((b >> i) & 1) ? 0.5 : -0.5;
            else f = (((b >> i) ^ (b >> j)) & 1) ? -0.25 : 0.25;
            acc[p] += f * w;
        }
    }
    __shared__ double red[kThreads / 64][kGradChunk];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < kGradChunk; ++p) {
        if (p >= a.np) continue;
        const double s = wave_sum(acc[p]);
        if (lane == 0) red[wv][p] = s;
    }
    __syncthreads();
    if (threadIdx.x < a.np) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += red[w][threadIdx.x];
        a.slots[(size_t)blockIdx.x * a.stride + a.off + threadIdx.x] += a.coef * s;
    }
}

// The same sums for every parameter of an axis at once.  Lane t of workgroup w takes the
// amplitudes b = w * 1024 + e * 64 + t, e < 16 (coalesced loads; index bits 6-9 vary along
// e, the others are fixed for the lane) and forms the Walsh sums
// M[m] = sum_e w_e prod_{k in m} s_{6+k}(b_e) of w = Im(conj(lam) psi) over the subsets m of
// those four bits (four butterfly stages: the sum without bit k, and half the difference
// for the subsets with it, s = +-1/2).  A parameter whose spins among bits 6-9 form the set
// m then gets M[m] times s_q of each of its other spins (fixed for the lane); the host groups
// the parameters by m so that M is indexed at compile time.  One wave reduction per
// parameter; lane 0 adds the workgroup's sum to its row of the slots.
template <typename R>
__global__ __launch_bounds__(kGradWalshBlock) void grad_walsh_kernel(const typename Vec<R>::T *__restrict__ psi,
                                                                   const typename Vec<R>::T *__restrict__ lam,
                                                                   GradWalshArgs a)
{
    using V = typename Vec<R>::T;
    constexpr int L = kGradWalshLow;
    const uint64_t base = (uint64_t)blockIdx.x * (kGradWalshBlock * kGradWalshElems) + threadIdx.x;
    double M[kGradWalshElems];
#pragma unroll
    for (int e = 0; e < kGradWalshElems; ++e) {
        const V u = psi[base + ((uint64_t)e << L)], l = lam[base + ((uint64_t)e << L)];
        M[e] = (double)l.x * (double)u.y - (double)l.y * (double)u.x;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int e = 0; e < kGradWalshElems; ++e)
            if (!(e & (1 << k))) {
                const double w0 = M[e], w1 = M[e | (1 << k)];
                M[e] = w0 + w1;
                M[e | (1 << k)] = 0.5 * (w1 - w0);
            }
    // every lane's Walsh sums into LDS (row m padded to 65 entries: rows with different m
    // fall in different banks); then lane p, one parameter per lane, sums the 64 lanes'
    // entries of its row m times the signs of its spins among the lane bits 0-5, and times
    // the signs of its spins at bits 10 and above (fixed for the workgroup)
    __shared__ double gm[kGradWalshElems * 65];
#pragma unroll
    for (int m = 0; m < kGradWalshElems; ++m) gm[m * 65 + threadIdx.x] = M[m];
    __syncthreads();
    const uint64_t wbase = (uint64_t)blockIdx.x * (kGradWalshBlock * kGradWalshElems);
    double *row = a.slots + (size_t)blockIdx.x * a.stride + a.off;
    for (int p = threadIdx.x; p < a.np; p += kGradWalshBlock) {
        const int i = a.pi[p], j = a.pj[p];
        int m = 0, li = -1, lj = -1;
        double s = 1.0;
        if (i < L) li = i;
        else if (i < L + 4) m |= 1 << (i - L);
        else s = ((wbase >> i) & 1) ? 0.5 : -0.5;
        if (j >= 0) {
            if (j < L) lj = j;
            else if (j < L + 4) m |= 1 << (j - L);
            else s *= ((wbase >> j) & 1) ? 0.5 : -0.5;
        }
        double acc = 0.0;
        for (int t = 0; t < kGradWalshBlock; ++t) {
            double f = gm[m * 65 + t];
            if (li >= 0) f *= ((t >> li) & 1) ? 0.5 : -0.5;
            if (lj >= 0) f *= ((t >> lj) & 1) ? 0.5 : -0.5;
            acc += f;
        }
        row[a.col[p]] += a.coef * s * acc;
    }
}

hipError_t launch_grad_walsh(int dtype, const void *psi, const void *lam, const GradWalshArgs &a,
                             hipStream_t s)
{
    if (a.n < 10 || a.np < 1) return hipErrorInvalidValue;
    const uint32_t nblocks = (uint32_t)(1ull << (a.n - 10));
    if (dtype == 0)
        hipLaunchKernelGGL((grad_walsh_kernel<double>), dim3(nblocks), dim3(kGradWalshBlock), 0, s,
                           static_cast<const double2 *>(psi), static_cast<const double2 *>(lam), a);
    else
        hipLaunchKernelGGL((grad_walsh_kernel<float>), dim3(nblocks), dim3(kGradWalshBlock), 0, s,
                           static_cast<const float2 *>(psi), static_cast<const float2 *>(lam), a);
    return hipGetLastError();
}

// out[c] = sum over workgroups (fixed order) of the accumulated slots.
__global__ __launch_bounds__(kThreads) void grad_finalize_kernel(const double *slots, int nblocks,
                                                                 int ncols, double *out)
{
    const int lane = threadIdx.x & 63;
    for (int c = (int)(blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6)); c < ncols;
         c += (int)(gridDim.x * (kThreads / 64))) {
        double s = 0.0;
        for (int b = lane; b < nblocks; b += 64) s += slots[(size_t)b * ncols + c];
        s = wave_sum(s);
        if (lane == 0) out[c] = s;
    }
}

// ------------------------------------------------------------------------ launchers

hipError_t launch_batch_reduce(int dtype, const BatchReduceArgs &a, int nchains, double *partials,
                               int nbpc, hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL((batch_reduce_kernel<double>), dim3(nbpc, nchains), dim3(kThreads), 0, s, a,
                           partials);
    else
        hipLaunchKernelGGL((batch_reduce_kernel<float>), dim3(nbpc, nchains), dim3(kThreads), 0, s, a,
                           partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(nchains), dim3(kThreads), 0, s, a, partials, nbpc);
    return hipGetLastError();
}

hipError_t launch_apply_obs(int dtype, const void *psi, void *out, int kind, int i, int j, int n,
                            hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    uint64_t nb = (dim + kThreads - 1) / kThreads;
    if (nb > 4096) nb = 4096;
    if (dtype == 0)
        hipLaunchKernelGGL((apply_obs_kernel<double>), dim3((uint32_t)nb), dim3(kThreads), 0, s,
                           static_cast<const double2 *>(psi), static_cast<double2 *>(out), kind, i, j, n);
    else
        hipLaunchKernelGGL((apply_obs_kernel<float>), dim3((uint32_t)nb), dim3(kThreads), 0, s,
                           static_cast<const float2 *>(psi), static_cast<float2 *>(out), kind, i, j, n);
    return hipGetLastError();
}

hipError_t launch_apply_ham(int dtype, const void *psi, void *out, int n, const double *ham_h,
                            const HamBond *ham_b, int nb, hipStream_t s)
{
    const uint64_t dim = 1ull << n;
    uint64_t nblk = (dim + kThreads - 1) / kThreads;
    if (nblk > 4096) nblk = 4096;
    if (dtype == 0)
        hipLaunchKernelGGL((apply_ham_kernel<double>), dim3((uint32_t)nblk), dim3(kThreads), 0, s,
                           static_cast<const double2 *>(psi), static_cast<double2 *>(out), n, ham_h,
                           ham_b, nb);
    else
        hipLaunchKernelGGL((apply_ham_kernel<float>), dim3((uint32_t)nblk), dim3(kThreads), 0, s,
                           static_cast<const float2 *>(psi), static_cast<float2 *>(out), n, ham_h,
                           ham_b, nb);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(int dtype, const void *psi, const void *lam, const GradArgs &a,
                              int nblocks, hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL((grad_reduce_kernel<double>), dim3(nblocks), dim3(kThreads), 0, s,
                           static_cast<const double2 *>(psi), static_cast<const double2 *>(lam), a);
    else
        hipLaunchKernelGGL((grad_reduce_kernel<float>), dim3(nblocks), dim3(kThreads), 0, s,
                           static_cast<const float2 *>(psi), static_cast<const float2 *>(lam), a);
    return hipGetLastError();
}

hipError_t launch_grad_finalize(const double *slots, int nblocks, int ncols, double *out, hipStream_t s)
{
    const int per = kThreads / 64;
    const int grid = (ncols + per - 1) / per;
    hipLaunchKernelGGL(grad_finalize_kernel, dim3(grid), dim3(kThreads), 0, s, slots, nblocks, ncols, out);
    return hipGetLastError();
}

template <typename R, int T>
static hipError_t launch_sweep_t(void *psi, const SweepArgs &a, uint32_t nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_kernel<R, T>), dim3(nblocks), dim3(kThreads), 0, s,
                       reinterpret_cast<typename Vec<R>::T *>(psi), a);
    return hipGetLastError();
}

hipError_t launch_sweep(int dtype, int T, void *psi, const SweepArgs &a, uint32_t nblocks,
                        hipStream_t s)
{
#define TS_SW_CASE(TT) \
    case TT: return dtype == 0 ? launch_sweep_t<double, TT>(psi, a, nblocks, s) \
                               : launch_sweep_t<float, TT>(psi, a, nblocks, s);
    switch (T) {
        TS_SW_CASE(8)
        TS_SW_CASE(9)
        TS_SW_CASE(10)
        TS_SW_CASE(11)
        TS_SW_CASE(12)
        TS_SW_CASE(13)
    case 14:
        if (dtype == 1) return launch_sweep_t<float, 14>(psi, a, nblocks, s);
        break;
    default: break;
    }
#undef TS_SW_CASE
    return hipErrorInvalidValue;
}

// One workgroup per tile.
template <typename R, int T, int RB>
static hipError_t launch_reg_t(void *psi, const RegSweepArgs &a, uint64_t grid, hipStream_t s)
{
    hipLaunchKernelGGL((sweep_reg_kernel<R, T, RB>), dim3((uint32_t)grid), dim3(1 << (T - RB)),
                       0, s, reinterpret_cast<typename Vec<R>::T *>(psi), a);
    return hipGetLastError();
}

static hipError_t launch_reg_any(int dtype, int T, int RB, void *psi, const RegSweepArgs &a,
                                 uint64_t grid, hipStream_t s)
{
    if (grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
#define TS_RG_CASE(TT, RR)                                                                        \
    if (T == TT && RB == RR)                                                                      \
        return dtype == 0 ? launch_reg_t<double, TT, RR>(psi, a, grid, s)                         \
                          : launch_reg_t<float, TT, RR>(psi, a, grid, s);
    TS_RG_CASE(8, 4)
    TS_RG_CASE(9, 4)
    TS_RG_CASE(10, 4)
    TS_RG_CASE(11, 4)
    TS_RG_CASE(12, 4)
    TS_RG_CASE(13, 4)
    TS_RG_CASE(8, 3)
    TS_RG_CASE(9, 3)
    TS_RG_CASE(10, 3)
    TS_RG_CASE(11, 3)
    TS_RG_CASE(12, 3)
    TS_RG_CASE(13, 3)
    if (T == 14 && RB == 4 && dtype == 1) return launch_reg_t<float, 14, 4>(psi, a, grid, s);
#undef TS_RG_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_reg(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s)
{
    if (a.chains) return hipErrorInvalidValue;
    return launch_reg_any(dtype, T, RB, psi, a, a.psi2 ? 2 * a.n_tiles : a.n_tiles, s);
}

hipError_t launch_sweep_half(int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s)
{
    if (a.chains) return hipErrorInvalidValue;
    const uint64_t grid = a.psi2 ? 2 * a.n_tiles : a.n_tiles;
    if (grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
#define TS_HALF_CASE(TT, RR)                                                                        \
    if (T == TT && RB == RR) {                                                                      \
        hipLaunchKernelGGL((sweep_half_kernel<TT, RR>), dim3((uint32_t)grid), dim3(1 << (TT - RR)), \
                           0, s, static_cast<double2 *>(psi), a);                                   \
        return hipGetLastError();                                                                   \
    }
    TS_HALF_CASE(11, 4)
    TS_HALF_CASE(12, 4)
#undef TS_HALF_CASE
    return hipErrorInvalidValue;
}

// Resident workgroups of one pipelined sweep instance: CUs x blocks per CU, cached.
template <typename R, int T, int RB>
static hipError_t launch_pipe_t(void *psi, const RegSweepArgs &a, hipStream_t s)
{
    static int resident = 0;
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_pipe_kernel<R, T, RB>,
                                                             1 << (T - RB), 0);
        if (e != hipSuccess) return e;
        if (cus <= 0 || per_cu <= 0) return hipErrorInvalidConfiguration;
        resident = cus * per_cu;
    }
    const uint64_t grid = a.n_tiles < (uint64_t)resident ? a.n_tiles : (uint64_t)resident;
    if (grid == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sweep_pipe_kernel<R, T, RB>), dim3((uint32_t)grid), dim3(1 << (T - RB)), 0,
                       s, reinterpret_cast<typename Vec<R>::T *>(psi), a);
    return hipGetLastError();
}

hipError_t launch_sweep_pipe(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s)
{
    if (a.chains) return hipErrorInvalidValue;
#define TS_PIPE_CASE(TT, RR)                                                                      \
    if (T == TT && RB == RR)                                                                      \
        return dtype == 0 ? launch_pipe_t<double, TT, RR>(psi, a, s) : launch_pipe_t<float, TT, RR>(psi, a, s);
    // two register sets must fit without spills: tiles up to 2^12 (2^13 for complex64 with
    // eight amplitudes per thread)
    TS_PIPE_CASE(10, 4)
    TS_PIPE_CASE(10, 3)
    TS_PIPE_CASE(11, 4)
    TS_PIPE_CASE(11, 3)
    TS_PIPE_CASE(12, 4)
    TS_PIPE_CASE(12, 3)
    if (T == 13 && RB == 3 && dtype == 1) return launch_pipe_t<float, 13, 3>(psi, a, s);
#undef TS_PIPE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_sweep_reg_batch(int dtype, int T, int RB, const RegSweepArgs &a, uint32_t nchains,
                                  hipStream_t s)
{
    if (!a.chains || a.tiles_per_chain == 0) return hipErrorInvalidValue;
    return launch_reg_any(dtype, T, RB, nullptr, a, (uint64_t)nchains * a.tiles_per_chain, s);
}

template <typename R, int T>
static hipError_t launch_res_t(const ResidentArgs &a, int nvec, hipStream_t s)
{
    hipLaunchKernelGGL((resident_kernel<R, T>), dim3(nvec), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_resident(int dtype, int T, const ResidentArgs &a, int nvec, hipStream_t s)
{
#define TS_RES_CASE(TT) \
    case TT: return dtype == 0 ? launch_res_t<double, TT>(a, nvec, s) : launch_res_t<float, TT>(a, nvec, s);
    switch (T) {
        TS_RES_CASE(8)
        TS_RES_CASE(9)
        TS_RES_CASE(10)
        TS_RES_CASE(11)
        TS_RES_CASE(12)
        TS_RES_CASE(13)
    case 14:
        if (dtype == 1) return launch_res_t<float, 14>(a, nvec, s);
        break;
    default: break;
    }
#undef TS_RES_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_resident_factors(int T, const ResidentArgs &a, double2 *out, hipStream_t s)
{
    if (a.chains || a.n_ops <= 0 || a.n > T) return hipErrorInvalidValue;
#define TS_RESF_CASE(TT)                                                                                 \
    case TT:                                                                                             \
        hipLaunchKernelGGL((resident_factor_kernel<TT>), dim3((uint32_t)a.n_ops), dim3(kThreads), 0, s, a, \
                           out);                                                                         \
        return hipGetLastError();
    switch (T) {
        TS_RESF_CASE(8)
        TS_RESF_CASE(9)
        TS_RESF_CASE(10)
        TS_RESF_CASE(11)
        TS_RESF_CASE(12)
        TS_RESF_CASE(13)
    default: break;
    }
#undef TS_RESF_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_reduce(int dtype, const ReduceArgs &a, double *partials, int nblocks,
                         double *out, hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL((reduce_kernel<double>), dim3(nblocks), dim3(kThreads), 0, s, a, partials);
    else
        hipLaunchKernelGGL((reduce_kernel<float>), dim3(nblocks), dim3(kThreads), 0, s, a, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s, partials, nblocks, a, out);
    return hipGetLastError();
}

// The fixed scratch: one copy per GPU.  In host code `scratch` names a host-side stand-in,
// not device memory, so every host use goes through the address hipGetSymbolAddress returns.
static __device__ __align__(256) double scratch[kScratchDoubles];

hipError_t scratch_address(double **out)
{
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<double *>(p);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_sweep_etab(int dtype, int T, int RB, void *psi, const RegSweepArgs &a, hipStream_t s)
{
    if ((RB != 3 && RB != 4) || a.n_tiles == 0 || a.n_tiles > 0x7fffffffull || a.chains) return hipErrorInvalidValue;
#define TS_ETAB_CASE(TT, RR)                                                                      \
    if (T == TT && RB == RR) {                                                                    \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((sweep_etab_kernel<double, TT, RR>), dim3((uint32_t)a.n_tiles),     \
                               dim3(1 << (TT - RR)), 0, s, static_cast<double2 *>(psi), a);       \
        else                                                                                      \
            hipLaunchKernelGGL((sweep_etab_kernel<float, TT, RR>), dim3((uint32_t)a.n_tiles),      \
                               dim3(1 << (TT - RR)), 0, s, static_cast<float2 *>(psi), a);        \
        return hipGetLastError();                                                                 \
    }
    TS_ETAB_CASE(8, 4)
    TS_ETAB_CASE(9, 4)
    TS_ETAB_CASE(10, 4)
    TS_ETAB_CASE(11, 4)
    TS_ETAB_CASE(12, 4)
    TS_ETAB_CASE(13, 4)
    TS_ETAB_CASE(8, 3)
    TS_ETAB_CASE(9, 3)
    TS_ETAB_CASE(10, 3)
    TS_ETAB_CASE(11, 3)
    TS_ETAB_CASE(12, 3)
    TS_ETAB_CASE(13, 3)
#undef TS_ETAB_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_energy_table(int dtype, void *out, int n, const double *h, const HamBond *bonds, int n_bonds,
                               int axis, hipStream_t s)
{
    if (!out || !h || (n_bonds > 0 && !bonds) || n < 1 || n > 40 || axis < 0 || axis > 2)
        return hipErrorInvalidValue;
    const uint64_t count = 1ull << n;
    const uint64_t blocks = std::min<uint64_t>((count + kThreads - 1) / kThreads, 1u << 16);
    if (dtype == 0)
        hipLaunchKernelGGL(energy_table_kernel<double>, dim3((uint32_t)blocks), dim3(kThreads), 0, s,
                           static_cast<double *>(out), n, h, bonds, n_bonds, axis, count);
    else
        hipLaunchKernelGGL(energy_table_kernel<float>, dim3((uint32_t)blocks), dim3(kThreads), 0, s,
                           static_cast<float *>(out), n, h, bonds, n_bonds, axis, count);
    return hipGetLastError();
}

hipError_t launch_sweep_pair(int dtype, int T, int RB, void *psi, void *lam, const RegSweepArgs &a,
                             const PairGradArgs &g, hipStream_t s)
{
    if (RB != 4 || a.n_tiles == 0 || a.n_tiles > 0x7fffffffull) return hipErrorInvalidValue;
#define TS_PAIR_CASE(TT)                                                                          \
    if (T == TT) {                                                                                \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((sweep_pair_kernel<double, TT, 4>), dim3((uint32_t)a.n_tiles),      \
                               dim3(1 << (TT - 4)), 0, s, static_cast<double2 *>(psi),             \
                               static_cast<double2 *>(lam), a, g);                                \
        else                                                                                      \
            hipLaunchKernelGGL((sweep_pair_kernel<float, TT, 4>), dim3((uint32_t)a.n_tiles),       \
                               dim3(1 << (TT - 4)), 0, s, static_cast<float2 *>(psi),              \
                               static_cast<float2 *>(lam), a, g);                                 \
        return hipGetLastError();                                                                 \
    }
    TS_PAIR_CASE(8)
    TS_PAIR_CASE(9)
    TS_PAIR_CASE(10)
    TS_PAIR_CASE(11)
    TS_PAIR_CASE(12)
#undef TS_PAIR_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_cone(int dtype, int T, int RB, void *psi, const ConeArgs *a, int n_phases,
                       uint64_t n_tiles, int reverse, hipStream_t s)
{
    if (!a || RB != 4 || n_phases < 0 || n_phases > kConePhases || n_tiles == 0 || n_tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
#define TS_CONE_CASE(TT)                                                                          \
    if (T == TT) {                                                                                \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((cone_c128_kernel<TT, 4>), dim3((uint32_t)n_tiles), dim3(1 << (TT - 4)), \
                               0, s, static_cast<double2 *>(psi), a, n_tiles, reverse);        \
        else                                                                                      \
            hipLaunchKernelGGL((cone_c64_kernel<TT, 4>), dim3((uint32_t)n_tiles), dim3(1 << (TT - 4)), \
                               0, s, static_cast<float2 *>(psi), a, n_tiles, reverse);         \
        return hipGetLastError();                                                                 \
    }
    TS_CONE_CASE(11)
    TS_CONE_CASE(12)
#undef TS_CONE_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_cone_rec(int dtype, int T, int RB, void *psi, const ConeArgs *a, int n_phases,
                           uint64_t n_tiles, int reverse, const ConeRec &rec, hipStream_t s)
{
    if (!a || !rec.partials || RB != 4 || n_phases < 0 || n_phases > kConePhases || n_tiles == 0 ||
        n_tiles > 0x7fffffffull || rec.n_obs < 0 || rec.n_obs > kConeRecMax)
        return hipErrorInvalidValue;
#define TS_CONER_CASE(TT)                                                                         \
    if (T == TT) {                                                                                \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((cone_rec_c128_kernel<TT, 4>), dim3((uint32_t)n_tiles),             \
                               dim3(1 << (TT - 4)), 0, s, static_cast<double2 *>(psi), a, n_tiles, \
                               reverse, rec);                                                     \
        else                                                                                      \
            hipLaunchKernelGGL((cone_rec_c64_kernel<TT, 4>), dim3((uint32_t)n_tiles),              \
                               dim3(1 << (TT - 4)), 0, s, static_cast<float2 *>(psi), a, n_tiles,  \
                               reverse, rec);                                                     \
        return hipGetLastError();                                                                 \
    }
    TS_CONER_CASE(11)
    TS_CONER_CASE(12)
#undef TS_CONER_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_cone_pair(int dtype, int T, int RB, void *psi, void *lam, const ConeArgs *a, int n_phases,
                            const ConeGradArgs *g, int n_slots, double *slots, int stride, uint64_t n_tiles,
                            int reverse, hipStream_t s)
{
    if (!a || !g || !slots || RB != 4 || n_phases < 0 || n_phases > kConePhases || n_slots < 0 ||
        n_slots > kConeGradSlots || n_tiles == 0 || n_tiles > 0x7fffffffull)
        return hipErrorInvalidValue;
#define TS_CONEP_CASE(TT)                                                                         \
    if (T == TT) {                                                                                \
        const size_t dyn = cone_tab_bytes<TT, 4>(n_phases) + (size_t)n_slots * 64 * sizeof(double); \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((cone_pair_c128_kernel<TT, 4>), dim3((uint32_t)n_tiles),            \
                               dim3(1 << (TT - 4)), dyn, s, static_cast<double2 *>(psi),           \
                               static_cast<double2 *>(lam), a, g, slots, stride, n_tiles, reverse); \
        else                                                                                      \
            hipLaunchKernelGGL((cone_pair_c64_kernel<TT, 4>), dim3((uint32_t)n_tiles),             \
                               dim3(1 << (TT - 4)), dyn, s, static_cast<float2 *>(psi),            \
                               static_cast<float2 *>(lam), a, g, slots, stride, n_tiles, reverse); \
        return hipGetLastError();                                                                 \
    }
    TS_CONEP_CASE(11)
    TS_CONEP_CASE(12)
#undef TS_CONEP_CASE
    return hipErrorInvalidValue;
}

// First pass of a long finalize: workgroup g sums rows [g * 1024, (g + 1) * 1024) of every
// used column into row g of tmp (a fixed order: per thread, then a wave and an LDS tree).
__global__ __launch_bounds__(kThreads) void partial_rows_kernel(const double *partials, int nrows,
                                                                int ncols, double *tmp)
{
    __shared__ double red[kThreads / 64];
    const int r0 = blockIdx.x * 1024, r1 = min(nrows, r0 + 1024);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int c = 0; c < ncols; ++c) {
        double acc = 0.0;
        for (int r = r0 + (int)threadIdx.x; r < r1; r += kThreads) acc += partials[(size_t)r * (2 * kMaxObs) + c];
        acc = wave_sum(acc);
        if (lane == 0) red[wv] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            double sum = 0.0;
            for (int w = 0; w < kThreads / 64; ++w) sum += red[w];
            tmp[(size_t)blockIdx.x * (2 * kMaxObs) + c] = sum;
        }
        __syncthreads();
    }
}

hipError_t launch_finalize(const double *partials, int nblocks, const ReduceArgs &a, double *out,
                           double *tmp, hipStream_t s)
{
    if (nblocks > 1024) {
        const int groups = (nblocks + 1023) / 1024;
        if (groups > 1024 || !tmp) return hipErrorInvalidValue;
        hipLaunchKernelGGL(partial_rows_kernel, dim3(groups), dim3(kThreads), 0, s, partials, nblocks,
                           2 * a.n_obs, tmp);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        partials = tmp;
        nblocks = groups;
    }
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kThreads), 0, s, partials, nblocks, a, out);
    return hipGetLastError();
}

hipError_t launch_cone_batch(int dtype, int T, int RB, void *packed, const int64_t *off,
                             const ConeArgs *args, uint32_t nchains, uint64_t tiles_per_chain, int reverse,
                             hipStream_t s)
{
    const uint64_t grid = (uint64_t)nchains * tiles_per_chain;
    if (!packed || !off || !args || RB != 4 || grid == 0 || grid > 0x7fffffffull) return hipErrorInvalidValue;
#define TS_CONEB_CASE(TT)                                                                         \
    if (T == TT) {                                                                                \
        if (dtype == 0)                                                                           \
            hipLaunchKernelGGL((cone_batch_kernel<double, TT, 4>), dim3((uint32_t)grid),           \
                               dim3(1 << (TT - 4)), 0, s,                                         \
                               static_cast<double2 *>(packed), off, args, tiles_per_chain, reverse); \
        else                                                                                      \
            hipLaunchKernelGGL((cone_batch_kernel<float, TT, 4>), dim3((uint32_t)grid),            \
                               dim3(1 << (TT - 4)), 0, s,                                         \
                               static_cast<float2 *>(packed), off, args, tiles_per_chain, reverse); \
        return hipGetLastError();                                                                 \
    }
    TS_CONEB_CASE(11)
    TS_CONEB_CASE(12)
#undef TS_CONEB_CASE
    return hipErrorInvalidValue;
}

}  // namespace tsk

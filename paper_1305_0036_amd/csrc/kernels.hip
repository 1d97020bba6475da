// kernels.hip -- gfx950 device code of libtsspin.
//
// Three kernel families:
//   sweep_kernel     one pass over a state vector larger than a tile.  Each workgroup owns
//                    one closed set of 2^T amplitudes (Sec. 3.3: fixing the spins outside a
//                    group leaves a set closed under flipping the spins inside it), stages
//                    it in LDS, applies [butterflies on the group's bits] [phase step]
//                    [butterflies on the same bits] and writes it back.  The low bits of
//                    the index always stay inside the tile, so each workgroup moves
//                    contiguous runs (Sec. 3.4).  The phase is fused with the rotations
//                    (Sec. 3.1: phase correction merged into the rotation pass).
//   resident_kernel  the same operations for a state that fits one tile, for a whole
//                    recording segment at once; one workgroup per state vector.
//   reduce_kernel    FP64 observables of Sec. 4.2 (norm, magnetisation, overlaps).
//
// Phase step.  The energy of axis a is D(b) = sum_j h_j s_j + sum_(i,j) J_ij s_i s_j with
// s = +-1/2 (Sec. 2, Eqs. 1 and ZZ-Phases).  It is split by who owns which bits:
//   workgroup  fixes the bits outside the tile: a host table holds, per workgroup, the
//              energy of those bits (C) and the effective field they put on each tile bit
//              (geff); the tile-internal couplings are a T x T matrix.
//   thread     fixes tile bits 0..7 (its lane index within the 256-thread workgroup) and
//              owns the 2^(T-8) amplitudes that differ in tile bits 8..T-1.
//   element    adds the var-bit fields (a Gray-code walk of phase factors) and the var-var
//              couplings (a per-launch table in LDS).
// The argument reduction and every phase factor are FP64 for both storage precisions.
#include <hip/hip_runtime.h>
#include <stdint.h>

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

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
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

__device__ __forceinline__ void apply_phase(double2 &x, double2 z) { x = cmul(x, z); }
__device__ __forceinline__ void apply_phase(float2 &x, double2 z)
{
    const float zr = (float)z.x, zi = (float)z.y;
    const float xr = x.x, xi = x.y;
    x.x = xr * zr - xi * zi;
    x.y = xr * zi + xi * zr;
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

// Whole-state kernel: one workgroup per vector runs every (phase, layer) pass of a segment.
// For n < 8 the T = 8 instance is used with only 2^n amplitudes live.
template <typename R, int T>
__global__ __launch_bounds__(kThreads) void resident_kernel(ResidentArgs a)
{
    using V = typename Vec<R>::T;
    constexpr int NV = T - kFixedBits;
    __shared__ V tile[1 << T];
    __shared__ double2 qtab[1 << NV];
    V *psi = reinterpret_cast<V *>(a.psi[blockIdx.x]);
    const int ne = 1 << a.n;
    for (int t = threadIdx.x; t < ne; t += kThreads) tile[t] = psi[t];
    __syncthreads();
    const uint32_t all = (uint32_t)(ne - 1);
    for (int s = 0; s < a.n_ops; ++s) {
        const ResidentOp op = a.ops[s];
        if (op.d.axis >= 0) {
            const int ax = op.d.axis < 3 ? op.d.axis : 0;
            build_qtab<T>(qtab, op.d, a.jt[ax]);
            __syncthreads();
            diag_step<T>(tile, ne, op.d, a.wg[ax], a.jt[ax], qtab, (uint64_t)threadIdx.x);
            __syncthreads();
        }
        if (op.post) wht_layer(tile, ne, all);
    }
    for (int t = threadIdx.x; t < ne; t += kThreads) psi[t] = tile[t];
}

// ----------------------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
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

// Sum the per-block partials in a fixed order and write the requested slots.
__global__ void finalize_kernel(const double *partials, int nblocks, ReduceArgs a, double *out)
{
    const int s = threadIdx.x;
    if (s >= 2 * a.n_obs) return;
    double acc = 0.0, comp = 0.0;
    for (int b = 0; b < nblocks; ++b) {  // Neumaier-compensated
        const double x = partials[(size_t)b * (2 * kMaxObs) + s];
        const double t = acc + x;
        comp += (fabs(acc) >= fabs(x)) ? (acc - t) + x : (x - t) + acc;
        acc = t;
    }
    const int o = s >> 1, part = s & 1;
    const ObsDev ob = a.obs[o];
    if (part == 1 && ob.kind != 7) return;
    out[ob.slot + part] = acc + comp;
}

// ------------------------------------------------------------------------ launchers

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

hipError_t launch_reduce(int dtype, const ReduceArgs &a, double *partials, int nblocks,
                         double *out, hipStream_t s)
{
    if (dtype == 0)
        hipLaunchKernelGGL((reduce_kernel<double>), dim3(nblocks), dim3(kThreads), 0, s, a, partials);
    else
        hipLaunchKernelGGL((reduce_kernel<float>), dim3(nblocks), dim3(kThreads), 0, s, a, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, s, partials, nblocks, a, out);
    return hipGetLastError();
}

}  // namespace tsk

// Device helpers shared by the kernel files: wavefront/block reductions with a
// deterministic last-block finish, packed-table lookups, SplitMix64.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace hphi {

constexpr int kBlock = 256;      // threads per workgroup for streaming kernels
constexpr int kWave = 64;

// complex FP64 arithmetic of the shifted COCG
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cadd(cd a, cd b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cd csub(cd a, cd b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cd cdiv(cd a, cd b)
{
    // Smith's algorithm
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, d = b.re + b.im * r;
        return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
    }
    const double r = b.re / b.im, d = b.re * r + b.im;
    return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ double cabs2(cd a) { return a.re * a.re + a.im * a.im; }

// COCG scalar step once mu = p^T (z_s p - H p) is known: alpha = rho / mu
// (breakdown when mu = 0). One thread.
__device__ __forceinline__ void cocg_alpha_step(CgDev *cg, cd mu)
{
    cg->alpha_prev = cg->alpha;
    cg->beta_prev = cg->beta;
    if (cabs2(mu) == 0.0) {
        cg->breakdown = 1;
        cg->alpha = {0.0, 0.0};
    } else {
        cg->alpha = cdiv(cg->rho, mu);
    }
    __threadfence();
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Reduce NR per-thread values over the block; on return thread 0 holds the
// sums in vals[]. `sh` needs NR * (blockDim / 64) doubles.
template <int NR>
__device__ __forceinline__ void block_sum(double (&vals)[NR], double *sh)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NR; ++i) vals[i] = wave_sum(vals[i]);
    __syncthreads();
    if (lane == 0)
        for (int i = 0; i < NR; ++i) sh[i * nw + wid] = vals[i];
    __syncthreads();
    if (threadIdx.x == 0)
        for (int i = 0; i < NR; ++i) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sh[i * nw + w];
            vals[i] = s;
        }
    __syncthreads();
}

// Block partials -> red.partial[block * nres + i]; the last block to finish
// sums the partials of all blocks in block order (fixed order, hence
// run-to-run identical) into red.result[i] and re-arms the counter.
// Returns true in the last block (all threads) so callers can finish scalar
// work after the reduction; red.result is then valid for thread 0 only after
// the final __syncthreads inside.
// `last` is a block-shared flag word (static LDS in grid_finish; kernels
// that keep all of their LDS dynamic pass one of their own).
__device__ __forceinline__ bool grid_finish_at(const double *blockvals, int nres, const Reduce &red,
                                               double *sh, unsigned *last)
{
    if (threadIdx.x == 0) {
        for (int i = 0; i < nres; ++i) red.partial[(size_t)blockIdx.x * nres + i] = blockvals[i];
        __threadfence();
        unsigned prev = atomicAdd(red.counter, 1u);
        *last = (prev == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!*last) return false;
    __threadfence();
    const int nb = gridDim.x;
    for (int i = 0; i < nres; ++i) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x)
            v += __builtin_nontemporal_load(&red.partial[(size_t)b * nres + i]);
        double vv[1] = {v};
        block_sum<1>(vv, sh);
        if (threadIdx.x == 0) red.result[i] = vv[0];
    }
    if (threadIdx.x == 0) *red.counter = 0u;
    __threadfence();
    __syncthreads();
    return true;
}

__device__ __forceinline__ bool grid_finish(const double *blockvals, int nres, const Reduce &red,
                                            double *sh)
{
    __shared__ unsigned s_last;
    return grid_finish_at(blockvals, nres, red, sh, &s_last);
}

// SplitMix64 (Steele, Lea, Flood 2014): state advances by the golden-ratio
// constant; output is the published finalizer of the state.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t i)
{
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ double u53(uint64_t z) { return (double)(z >> 11) * (1.0 / 9007199254740992.0); }

// Fused epilogue out = c1 * raw + c2 * u over K scalars of one state. Real
// coefficients (cplx = 0), or complex ones applied to (re, im) pairs
// (cplx = 1, K even): coef = [c1 re, c2 re, c1 im, c2 im]. u may be null.
template <typename S, int K>
__device__ __forceinline__ void epilogue(const S (&raw)[K], const S *uu, int cplx, const double *coef,
                                         S (&out)[K])
{
    const S c1r = coef ? (S)coef[0] : (S)1, c2r = coef ? (S)coef[1] : (S)0;
    if constexpr (K % 2 == 0) {
        if (cplx) {
            const S c1i = (S)coef[2], c2i = (S)coef[3];
#pragma unroll
            for (int k = 0; k < K; k += 2) {
                out[k] = c1r * raw[k] - c1i * raw[k + 1];
                out[k + 1] = c1r * raw[k + 1] + c1i * raw[k];
                if (uu) {
                    out[k] += c2r * uu[k] - c2i * uu[k + 1];
                    out[k + 1] += c2r * uu[k + 1] + c2i * uu[k];
                }
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        out[k] = c1r * raw[k];
        if (uu) out[k] += c2r * uu[k];
    }
}

// The same epilogue with u held in registers (has_u false: no u term);
// identical arithmetic, no pointer to a private array.
template <typename S, int K>
__device__ __forceinline__ void epilogue_r(const S (&raw)[K], const S (&uu)[K], bool has_u, int cplx,
                                           const double *coef, S (&out)[K])
{
    const S c1r = coef ? (S)coef[0] : (S)1, c2r = coef ? (S)coef[1] : (S)0;
    if constexpr (K % 2 == 0) {
        if (cplx) {
            const S c1i = (S)coef[2], c2i = (S)coef[3];
#pragma unroll
            for (int k = 0; k < K; k += 2) {
                out[k] = c1r * raw[k] - c1i * raw[k + 1];
                out[k + 1] = c1r * raw[k + 1] + c1i * raw[k];
                if (has_u) {
                    out[k] += c2r * uu[k] - c2i * uu[k + 1];
                    out[k + 1] += c2r * uu[k + 1] + c2i * uu[k];
                }
            }
            return;
        }
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        out[k] = c1r * raw[k];
        if (has_u) out[k] += c2r * uu[k];
    }
}

template <typename T> struct VecOf;
template <> struct VecOf<double> { using t2 = double2; };
template <> struct VecOf<float> { using t2 = float2; };

} // namespace hphi

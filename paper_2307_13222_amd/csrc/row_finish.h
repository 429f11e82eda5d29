// The caller's epilogue of one H*v output element and the per-lane FP64
// dot products, shared by the row-per-thread kernels of the models without
// a fused Lanczos update (SpinGC, spin-S):
//   out = c1 * hv + c2 * u  (real, or complex coefficients on (re, im)),
//   w = out; raw_out = hv; acc += out; dots <v, x> and <x, x> per lane with
//   x = hv (dot_raw) or out, summed over the wave, the block's waves in
//   order and the blocks by the deterministic last-block finish.
#pragma once

#include "kern_common.h"

namespace hphi {

template <typename S>
struct EpiArgs {
    S *w;
    const S *u;
    S *acc;
    S *raw;
    const double *coef;
    int coef_cplx;
    int dot_raw;
};

template <typename S, int NV, bool DOTS>
struct RowFinish {
    static constexpr int ND = DOTS ? NV : 1;
    double d0[ND], d1[ND];
    S c1s, c2s;

    __device__ __forceinline__ void init(const EpiArgs<S> &e)
    {
#pragma unroll
        for (int j = 0; j < ND; ++j) d0[j] = d1[j] = 0.0;
        c1s = e.coef ? (S)e.coef[0] : (S)1;
        c2s = e.coef ? (S)e.coef[1] : (S)0;
    }

    // hv: H v of the element at offset off (in elements of NV lanes); me: v there
    __device__ __forceinline__ void apply(const S (&hv)[NV], const S (&me)[NV], size_t off, const EpiArgs<S> &e)
    {
        S out[NV];
        if (e.coef_cplx) {
            S uu[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) uu[j] = e.u ? e.u[off * NV + j] : (S)0;
            epilogue_r<S, NV>(hv, uu, e.u != nullptr, 1, e.coef, out);
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j) out[j] = c1s * hv[j] + (e.u ? c2s * e.u[off * NV + j] : (S)0);
        }
#pragma unroll
        for (int j = 0; j < NV; ++j) e.w[off * NV + j] = out[j];
        if (e.raw) {
#pragma unroll
            for (int j = 0; j < NV; ++j) e.raw[off * NV + j] = hv[j];
        }
        if (e.acc) {
#pragma unroll
            for (int j = 0; j < NV; ++j) e.acc[off * NV + j] += out[j];
        }
        if constexpr (DOTS) {
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double o = e.dot_raw ? (double)hv[j] : (double)out[j];
                d0[j] += (double)me[j] * o;
                d1[j] += o * o;
            }
        }
    }

    // once per workgroup after its last element; sh_red: 2 NV doubles per
    // wave, sh_blk: 2 NV doubles
    __device__ __forceinline__ void reduce(const Reduce &red, double *sh_red, double *sh_blk)
    {
        if constexpr (DOTS) {
            const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                const double s0 = wave_sum(d0[j]), s1 = wave_sum(d1[j]);
                if (lane == 0) {
                    sh_red[wid * 2 * NV + j] = s0;
                    sh_red[wid * 2 * NV + NV + j] = s1;
                }
            }
            __syncthreads();
            if (tid < 2 * NV) {
                double s = 0.0;
                for (int w2 = 0; w2 < nw; ++w2) s += sh_red[w2 * 2 * NV + tid];
                sh_blk[tid] = s;
            }
            __syncthreads();
            grid_finish(sh_blk, 2 * NV, red, sh_red);
        }
    }
};

} // namespace hphi

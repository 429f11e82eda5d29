// Streaming vector kernels around the H*v: seeded start vectors, FP64 dots
// and norms with deterministic reductions, scaling and axpy, the fused
// Lanczos update, the basis rank/unrank kernels, the trace of H and the
// S^z(q) excitation.
#include "kern_common.h"
#include "hub_pairs.h"

namespace hphi {

template <typename S> __device__ __forceinline__ S *P(void *p) { return static_cast<S *>(p); }
template <typename S> __device__ __forceinline__ const S *P(const void *p) { return static_cast<const S *>(p); }

static int grid_for(int64_t n, int per_thread = 4)
{
    int64_t g = (n + (int64_t)kBlock * per_thread - 1) / ((int64_t)kBlock * per_thread);
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

// ---------------------------------------------------------------- random --
template <typename S>
__global__ void k_rng_uniform(S *out, int64_t n, uint64_t seed)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (S)(u53(splitmix64_at(seed, (uint64_t)i)) - 0.5);
}

// Element (r, j) of an interleaved block of complex vectors: vector j uses
// seed + j; its element r is sqrt(-2 ln u1) e^{2 pi i u2} (Box-Muller) with
// u1 = 1 - U(2r), u2 = U(2r + 1) from that vector's SplitMix64 stream.
template <typename S>
__global__ void k_rng_cgauss(S *out, int64_t dim, int nvec, uint64_t seed)
{
    const int64_t n = dim * nvec;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / nvec;
        const int j = (int)(t - r * nvec);
        const uint64_t sd = seed + (uint64_t)j;
        const double u1 = 1.0 - u53(splitmix64_at(sd, 2 * (uint64_t)r));
        const double u2 = u53(splitmix64_at(sd, 2 * (uint64_t)r + 1));
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincospi(2.0 * u2, &sn, &cs);
        out[2 * t] = (S)(rad * cs);
        out[2 * t + 1] = (S)(rad * sn);
    }
}

int launch_rng_uniform(int dtype, void *out, int64_t n, uint64_t seed, hipStream_t st)
{
    int g = grid_for(n);
    if (dtype_is_f32(dtype)) hipLaunchKernelGGL(k_rng_uniform<float>, dim3(g), dim3(kBlock), 0, st, (float *)out, n, seed);
    else hipLaunchKernelGGL(k_rng_uniform<double>, dim3(g), dim3(kBlock), 0, st, (double *)out, n, seed);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// The uniform stream laid out in rows of `cols` elements at pitch `ld`:
// element (r, c) is stream element r * cols + c; the padding is zero.
template <typename S>
__global__ void k_rng_uniform_pitched(S *out, int64_t rows, int64_t cols, int64_t ld, uint64_t seed)
{
    const int64_t n = rows * ld;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = t / ld, c = t - r * ld;
        out[t] = c < cols ? (S)(u53(splitmix64_at(seed, (uint64_t)(r * cols + c))) - 0.5) : (S)0;
    }
}

int launch_rng_uniform_pitched(int dtype, void *out, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                               hipStream_t st)
{
    int g = grid_for(rows * ld);
    if (dtype_is_f32(dtype))
        hipLaunchKernelGGL(k_rng_uniform_pitched<float>, dim3(g), dim3(kBlock), 0, st, (float *)out, rows, cols, ld, seed);
    else
        hipLaunchKernelGGL(k_rng_uniform_pitched<double>, dim3(g), dim3(kBlock), 0, st, (double *)out, rows, cols, ld,
                           seed);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// |x|^2 of a vector stored in rows of `cols` elements at pitch ld, summed in
// the order k_dots uses for the same vector unpadded (same grid, same
// element-to-thread assignment), so padded and unpadded runs agree bit for bit.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_norm2_pitched(const S *x, int64_t dim, int64_t cols, int64_t ld, Reduce red)
{
    __shared__ double sh[kBlock / kWave * 64];
    __shared__ double blk[64];
    double acc[1] = {0.0};
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const double a = (double)x[(r / cols) * ld + r % cols];
        acc[0] += a * a;
    }
    block_sum<1>(acc, sh);
    if (threadIdx.x == 0) blk[0] = acc[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

int launch_rng_cgauss(int dtype, void *out, int64_t dim, int nvec, uint64_t seed, hipStream_t st)
{
    int g = grid_for(dim * nvec);
    if (dtype_is_f32(dtype)) hipLaunchKernelGGL(k_rng_cgauss<float>, dim3(g), dim3(kBlock), 0, st, (float *)out, dim, nvec, seed);
    else hipLaunchKernelGGL(k_rng_cgauss<double>, dim3(g), dim3(kBlock), 0, st, (double *)out, dim, nvec, seed);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// ------------------------------------------------------------------ dots --
// Per-lane FP64 sums over rows of an interleaved block with `nl` lanes:
// mode 0: sum_r x[r, l] y[r, l]; mode 1: sum_r x[r, l]^2.
template <typename S, int NL>
__global__ __launch_bounds__(kBlock) void k_dots(const S *x, const S *y, int64_t rows, int mode, Reduce red)
{
    __shared__ double sh[kBlock / kWave * 64];
    __shared__ double blk[64];
    double acc[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) acc[l] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
            double a = (double)x[r * NL + l];
            acc[l] += mode == 0 ? a * (double)y[r * NL + l] : a * a;
        }
    }
    block_sum<NL>(acc, sh);
    if (threadIdx.x == 0)
        for (int l = 0; l < NL; ++l) blk[l] = acc[l];
    __syncthreads();
    grid_finish(blk, NL, red, sh);
}

template <typename S>
static int dots_t(int nl, int64_t rows, const void *x, const void *y, Reduce red, int mode, hipStream_t st)
{
    int g = grid_for(rows, 2);
#define DOTS_CASE(N) case N: hipLaunchKernelGGL((k_dots<S, N>), dim3(g), dim3(kBlock), 0, st, (const S *)x, (const S *)y, rows, mode, red); break;
    switch (nl) {
        DOTS_CASE(1) DOTS_CASE(2) DOTS_CASE(4) DOTS_CASE(8) DOTS_CASE(16) DOTS_CASE(32)
    default: return fail(HPHI_ERR_UNSUPPORTED, "dots: %d lanes", nl);
    }
#undef DOTS_CASE
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_dots(int dtype, int nlanes, int64_t rows, const void *x, const void *y, Reduce red,
                int mode, hipStream_t st)
{
    if (dtype_is_f32(dtype)) return dots_t<float>(nlanes, rows, x, y, red, mode, st);
    return dots_t<double>(nlanes, rows, x, y, red, mode, st);
}

int launch_norm2_pitched(int dtype, const void *x, int64_t dim, int64_t cols, int64_t ld, Reduce red, hipStream_t st)
{
    int g = grid_for(dim, 2);
    if (dtype_is_f32(dtype))
        hipLaunchKernelGGL(k_norm2_pitched<float>, dim3(g), dim3(kBlock), 0, st, (const float *)x, dim, cols, ld, red);
    else
        hipLaunchKernelGGL(k_norm2_pitched<double>, dim3(g), dim3(kBlock), 0, st, (const double *)x, dim, cols, ld, red);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// Per-lane x.y and y.y over flat [rows][NL] arrays: thread t always sees
// lane t % NL (the block size is a multiple of NL), so each thread keeps two
// FP64 sums; the block adds its threads of one lane in thread order, the
// last block adds the blocks' partials in block order.
template <typename S, int NL>
__global__ __launch_bounds__(kBlock) void k_dots_xy_yy(const S *x, const S *y, int64_t rows, Reduce red)
{
    __shared__ double sh[2 * kBlock];
    __shared__ double blk[2 * NL];
    __shared__ double shr[kBlock / kWave * 2];
    const int64_t n = rows * NL;
    double a0 = 0.0, a1 = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const double yv = (double)y[t];
        a0 += (double)x[t] * yv;
        a1 += yv * yv;
    }
    sh[threadIdx.x] = a0;
    sh[kBlock + threadIdx.x] = a1;
    __syncthreads();
    if (threadIdx.x < NL) {
        double s0 = 0.0, s1 = 0.0;
        for (int k = threadIdx.x; k < kBlock; k += NL) {
            s0 += sh[k];
            s1 += sh[kBlock + k];
        }
        blk[threadIdx.x] = s0;
        blk[NL + threadIdx.x] = s1;
    }
    __syncthreads();
    grid_finish(blk, 2 * NL, red, shr);
}

int launch_dots_xy_yy(int dtype, int nl, int64_t rows, const void *x, const void *y, Reduce red, hipStream_t st)
{
    if (nl < 1 || nl > 64 || kBlock % nl != 0) return fail(HPHI_ERR_UNSUPPORTED, "dots: %d lanes", nl);
    const int g = grid_for(rows * nl, 4);
    const bool f32 = dtype_is_f32(dtype);
#define XY_CASE(N)                                                                                             \
    case N:                                                                                                    \
        if (f32) hipLaunchKernelGGL((k_dots_xy_yy<float, N>), dim3(g), dim3(kBlock), 0, st, (const float *)x,  \
                                    (const float *)y, rows, red);                                              \
        else hipLaunchKernelGGL((k_dots_xy_yy<double, N>), dim3(g), dim3(kBlock), 0, st, (const double *)x,   \
                                (const double *)y, rows, red);                                                 \
        break;
    switch (nl) {
        XY_CASE(1) XY_CASE(2) XY_CASE(4) XY_CASE(8) XY_CASE(16) XY_CASE(32) XY_CASE(64)
    default: return fail(HPHI_ERR_UNSUPPORTED, "dots: %d lanes", nl);
    }
#undef XY_CASE
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// x[r, l] *= s[l] (mode 0) or 1/sqrt(s[l]) (mode 1); s per lane on device.
template <typename S>
__global__ void k_scale_lanes(S *x, int64_t rows, int nl, const double *s, int mode)
{
    const int64_t n = rows * nl;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int l = (int)(t % nl);
        const double f = mode == 0 ? s[l] : 1.0 / sqrt(s[l]);
        x[t] = (S)((double)x[t] * f);
    }
}

int launch_scale_lanes(int dtype, int nlanes, int64_t rows, void *x, const double *s, int mode,
                       hipStream_t st)
{
    int g = grid_for(rows * nlanes);
    if (dtype_is_f32(dtype)) hipLaunchKernelGGL(k_scale_lanes<float>, dim3(g), dim3(kBlock), 0, st, (float *)x, rows, nlanes, s, mode);
    else hipLaunchKernelGGL(k_scale_lanes<double>, dim3(g), dim3(kBlock), 0, st, (double *)x, rows, nlanes, s, mode);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// y += a x with a = a_dev[lane] (if a_dev) else a_host.
template <typename S>
__global__ void k_axpy_lanes(S *y, const S *x, int64_t rows, int nl, const double *a_dev, double a_host)
{
    const int64_t n = rows * nl;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double a = a_dev ? a_dev[t % nl] : a_host;
        y[t] = (S)((double)y[t] + a * (double)x[t]);
    }
}

int launch_axpy_lanes(int dtype, int nlanes, int64_t rows, void *y, const void *x, const double *a_dev,
                      double a_host, hipStream_t st)
{
    int g = grid_for(rows * nlanes);
    if (dtype_is_f32(dtype)) hipLaunchKernelGGL(k_axpy_lanes<float>, dim3(g), dim3(kBlock), 0, st, (float *)y, (const float *)x, rows, nlanes, a_dev, a_host);
    else hipLaunchKernelGGL(k_axpy_lanes<double>, dim3(g), dim3(kBlock), 0, st, (double *)y, (const double *)x, rows, nlanes, a_dev, a_host);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

template <typename D, typename S>
__global__ void k_copy_cast(D *d, const S *s, int64_t n)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x)
        d[t] = (D)s[t];
}

int launch_copy_cast(int dst_dtype, void *dst, int src_dtype, const void *src, int64_t n, hipStream_t st)
{
    int g = grid_for(n);
    const bool df = dtype_is_f32(dst_dtype), sf = dtype_is_f32(src_dtype);
    if (df && sf) hipLaunchKernelGGL((k_copy_cast<float, float>), dim3(g), dim3(kBlock), 0, st, (float *)dst, (const float *)src, n);
    else if (df) hipLaunchKernelGGL((k_copy_cast<float, double>), dim3(g), dim3(kBlock), 0, st, (float *)dst, (const double *)src, n);
    else if (sf) hipLaunchKernelGGL((k_copy_cast<double, float>), dim3(g), dim3(kBlock), 0, st, (double *)dst, (const float *)src, n);
    else hipLaunchKernelGGL((k_copy_cast<double, double>), dim3(g), dim3(kBlock), 0, st, (double *)dst, (const double *)src, n);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// --------------------------------------------------------------- Lanczos --
// Initial normalization bookkeeping: lz->nrm[0] holds |q_0|^2 (from k_dots);
// s_0 = 1/|q_0|, epilogue coefficients for the first H*v: c1 = s_0, c2 = 0.
__global__ void k_lz_init(LzDev *lz)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double n2 = lz->nrm[0];
        lz->s_cur = 1.0 / sqrt(n2);
        lz->s_prev = 0.0;
        lz->coef[0] = lz->s_cur;
        lz->coef[1] = 0.0;
        lz->iter = 0;
        lz->done = 0;
        lz->breakdown = 0;
    }
}

int launch_lz_init(int, LzDev *lz, int64_t, Reduce, hipStream_t st)
{
    hipLaunchKernelGGL(k_lz_init, dim3(1), dim3(64), 0, st, lz);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// After w = s_k H q_k - beta_k s_{k-1} q_{k-1} and lz->dot[0] = <q_k, w>:
//   alpha_k = s_k <q_k, w>;  w -= alpha_k s_k q_k;  beta_{k+1} = |w|;
// the last block stores alpha_k, beta_{k+1}, flags a breakdown
// (beta_{k+1} <= 1e-13 max(1, |alpha_k|)) and sets the next epilogue
// c1 = s_{k+1} = 1/beta_{k+1}, c2 = -beta_{k+1} s_k. q_{k+1} = w stays
// unnormalized; its scale s_{k+1} rides along in lz.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_lz_update(LzDev *lz, double *alpha, double *beta, int64_t dim,
                                                      S *__restrict__ w, const S *__restrict__ qk, Reduce red)
{
    __shared__ double sh[kBlock / kWave * 2];
    __shared__ double blk[1];
    if (lz->done) return;
    const double s = lz->s_cur;
    const double al = s * lz->dot[0];
    const double f = al * s;
    double acc = 0.0;
    // four independent rows per trip keep several loads in flight per wave
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; r + 3 * stride < dim; r += 4 * stride) {
        S wv[4], qv[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            wv[t] = w[r + t * stride];
            qv[t] = qk[r + t * stride];
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const S x = (S)((double)wv[t] - f * (double)qv[t]);
            w[r + t * stride] = x;
            acc += (double)x * (double)x;
        }
    }
    for (; r < dim; r += stride) {
        const S x = (S)((double)w[r] - f * (double)qk[r]);
        w[r] = x;
        acc += (double)x * (double)x;
    }
    double v[1] = {acc};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) blk[0] = v[0];
    __syncthreads();
    if (grid_finish(blk, 1, red, sh) && threadIdx.x == 0) {
        const double b = sqrt(red.result[0]);
        const int k = lz->iter;
        alpha[k] = al;
        beta[k + 1] = b;
        lz->iter = k + 1;
        if (!(b > 1e-13 * fmax(1.0, fabs(al)))) {
            lz->done = 1;
            lz->breakdown = 1;
        } else {
            lz->s_prev = s;
            lz->s_cur = 1.0 / b;
            lz->coef[0] = lz->s_cur;
            lz->coef[1] = -b * s;
        }
        __threadfence();
    }
}

int launch_lz_update(int dtype, LzDev *lz, double *alpha, double *beta, int64_t dim, void *w,
                     const void *qk, Reduce red, hipStream_t st)
{
    int g = grid_for(dim);
    if (dtype_is_f32(dtype)) hipLaunchKernelGGL(k_lz_update<float>, dim3(g), dim3(kBlock), 0, st, lz, alpha, beta, dim, (float *)w, (const float *)qk, red);
    else hipLaunchKernelGGL(k_lz_update<double>, dim3(g), dim3(kBlock), 0, st, lz, alpha, beta, dim, (double *)w, (const double *)qk, red);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// Second pass: psi += svec[k] * s_k * q_k (k = lz->iter before the update).
// psi += svec[k] s_k q_k; psi may be kept wider than q (P = double with
// FP32 storage: the Ritz vector of a refined solve).
// q may be stored in rows of `cols` elements at pitch ld (psi is not).
template <typename P, typename S>
__global__ void k_lz_psi(LzDev *lz, const double *svec, int64_t dim, P *psi, const S *qk, int64_t cols,
                         int64_t ld)
{
    if (lz->done) return;
    const double c = svec[lz->iter] * lz->s_cur;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t qr = ld == cols ? r : (r / cols) * ld + r % cols;
        psi[r] = (P)((double)psi[r] + c * (double)qk[qr]);
    }
}

int launch_lz_psi_accum(int psi_dtype, int dtype, LzDev *lz, const double *svec, int64_t dim, void *psi,
                        const void *qk, hipStream_t st, int64_t cols, int64_t ld)
{
    int g = grid_for(dim);
    if (cols <= 0) cols = ld = dim;
    const bool pf = dtype_is_f32(psi_dtype), qf = dtype_is_f32(dtype);
    if (pf && !qf) return fail(HPHI_ERR_INVALID_ARG, "Ritz vector narrower than the Krylov vectors");
    if (pf) hipLaunchKernelGGL((k_lz_psi<float, float>), dim3(g), dim3(kBlock), 0, st, lz, svec, dim, (float *)psi, (const float *)qk, cols, ld);
    else if (qf) hipLaunchKernelGGL((k_lz_psi<double, float>), dim3(g), dim3(kBlock), 0, st, lz, svec, dim, (double *)psi, (const float *)qk, cols, ld);
    else hipLaunchKernelGGL((k_lz_psi<double, double>), dim3(g), dim3(kBlock), 0, st, lz, svec, dim, (double *)psi, (const double *)qk, cols, ld);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// ----------------------------------------------------------------- basis --
struct SpecDev {
    const uint32_t *lo_rank;
    const uint64_t *hi_off;
    const uint32_t *lo_list;
    const uint32_t *lo_list_off;
    int n_bits, n_pop, n_lo, n_hi;
    int64_t dim;
};

static SpecDev spec_dev(const Species &s)
{
    SpecDev d;
    d.lo_rank = s.d_lo_rank.as<uint32_t>();
    d.hi_off = s.d_hi_off.as<uint64_t>();
    d.lo_list = s.d_lo_list.as<uint32_t>();
    d.lo_list_off = s.d_lo_list_off.as<uint32_t>();
    d.n_bits = s.n_bits;
    d.n_pop = s.n_pop;
    d.n_lo = s.n_lo;
    d.n_hi = s.n_hi;
    d.dim = s.dim;
    return d;
}

__device__ __forceinline__ int64_t dev_rank(const SpecDev &s, uint64_t x)
{
    if (s.n_bits < 64 && (x >> s.n_bits)) return -1;
    if (__popcll(x) != s.n_pop) return -1;
    const uint64_t lo = x & ((uint64_t(1) << s.n_lo) - 1);
    return (int64_t)(s.hi_off[x >> s.n_lo] + s.lo_rank[lo]);
}

// Unrank by binary search of hi_off (non-decreasing, 2^n_hi + 1 entries)
// for the last h with hi_off[h] <= r, then the lo pattern from the group
// of popcount n_pop - popcount(h).
__device__ __forceinline__ uint64_t dev_unrank(const SpecDev &s, int64_t r)
{
    int64_t lo = 0, hi = (int64_t(1) << s.n_hi);   // invariant hi_off[lo] <= r < hi_off[hi]
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (s.hi_off[mid] <= (uint64_t)r) lo = mid; else hi = mid;
    }
    const uint64_t h = (uint64_t)lo;
    const int k = s.n_pop - __popcll(h);
    const uint32_t l = s.lo_list[s.lo_list_off[k] + (uint32_t)((uint64_t)r - s.hi_off[h])];
    return (h << s.n_lo) | l;
}

__global__ void k_rank(SpecDev a, SpecDev b, int two, const uint64_t *x, int64_t n, int64_t *idx)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t s = x[t];
        if (!two) {
            idx[t] = dev_rank(a, s);
        } else {
            const int64_t ru = dev_rank(a, s >> 32), rd = dev_rank(b, s & 0xFFFFFFFFull);
            idx[t] = (ru < 0 || rd < 0) ? -1 : ru * b.dim + rd;
        }
    }
}

__global__ void k_unrank(SpecDev a, SpecDev b, int two, int64_t first, int64_t n, uint64_t *out)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = first + t;
        if (!two) {
            out[t] = dev_unrank(a, r);
        } else {
            const int64_t ru = r / b.dim, rd = r - ru * b.dim;
            out[t] = (dev_unrank(a, ru) << 32) | dev_unrank(b, rd);
        }
    }
}

template <typename T>
__global__ void k_materialize(SpecDev a, T *out)
{
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < a.dim;
         t += (int64_t)gridDim.x * blockDim.x)
        out[t] = (T)dev_unrank(a, t);
}

int launch_rank_device(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx, hipStream_t st)
{
    if (n <= 0) return HPHI_OK;
    SpecDev a = spec_dev(b->sp[0]);
    SpecDev c = b->kind == 1 ? spec_dev(b->sp[1]) : a;
    hipLaunchKernelGGL(k_rank, dim3(grid_for(n, 1)), dim3(kBlock), 0, st, a, c, b->kind, states, n, idx);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_states_device(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out, hipStream_t st)
{
    if (count <= 0) return HPHI_OK;
    SpecDev a = spec_dev(b->sp[0]);
    SpecDev c = b->kind == 1 ? spec_dev(b->sp[1]) : a;
    hipLaunchKernelGGL(k_unrank, dim3(grid_for(count, 1)), dim3(kBlock), 0, st, a, c, b->kind, first, count, out);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_materialize(Species &s, hipStream_t st)
{
    SpecDev a = spec_dev(s);
    int g = grid_for(s.dim, 1);
    if (s.state_bytes == 4) hipLaunchKernelGGL(k_materialize<uint32_t>, dim3(g), dim3(kBlock), 0, st, a, s.d_states.as<uint32_t>());
    else hipLaunchKernelGGL(k_materialize<uint64_t>, dim3(g), dim3(kBlock), 0, st, a, s.d_states.as<uint64_t>());
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// ----------------------------------------------------------------- trace --
__global__ __launch_bounds__(kBlock) void k_trace_spin(const uint32_t *states, int64_t dim,
                                                       const SpinBondDev *bonds, int nb,
                                                       const double *hz, int n_sites, Reduce red)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[1];
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = states[r];
        double d = 0.0;
        for (int b = 0; b < nb; ++b) {
            const uint32_t m = (uint32_t)bonds[b].mask, t = x & m;
            d += (t == 0u || t == m) ? bonds[b].jz4 : -bonds[b].jz4;
        }
        if (hz)
            for (int i = 0; i < n_sites; ++i) d -= hz[i] * (((x >> i) & 1u) ? 0.5 : -0.5);
        acc += d;
    }
    double v[1] = {acc};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) blk[0] = v[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

__global__ __launch_bounds__(kBlock) void k_trace_hub(const uint32_t *ups, const uint32_t *dns, int64_t dup,
                                                      int64_t ddn, const double *u_site, const HubPairDev *pairs,
                                                      int np, Reduce red)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[1];
    double acc = 0.0;
    const int64_t n = dup * ddn;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = ups[t / ddn], d = dns[t % ddn];
        uint32_t both = u & d;
        while (both) {
            acc += u_site[__builtin_ctz(both)];
            both &= both - 1u;
        }
        if (np) acc += hub_pair_diag(pairs, np, u, d);
    }
    double v[1] = {acc};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) blk[0] = v[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

// Double occupancy weight sum_x |psi_x|^2 * #(sites with both spins) of one
// complex vector (S = double or float, (re, im) interleaved), FP64 sum.
template <typename S>
__global__ __launch_bounds__(kBlock) void k_docc_hub(const uint32_t *ups, const uint32_t *dns, int64_t dup,
                                                     int64_t ddn, const S *psi, Reduce red)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[1];
    double acc = 0.0;
    const int64_t n = dup * ddn;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int nd = __builtin_popcount(ups[t / ddn] & dns[t % ddn]);
        const double re = (double)psi[2 * t], im = (double)psi[2 * t + 1];
        acc += (double)nd * (re * re + im * im);
    }
    double v[1] = {acc};
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) blk[0] = v[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

int launch_docc(hphi_ham *h, int dtype, const void *psi, Reduce red, hipStream_t st)
{
    const hphi_basis *b = h->basis;
    if (h->kind != 1) return fail(HPHI_ERR_UNSUPPORTED, "double occupancy is defined for Hubbard models");
    if (dtype == HPHI_C128)
        hipLaunchKernelGGL(k_docc_hub<double>, dim3(grid_for(b->dim, 4)), dim3(kBlock), 0, st,
                           b->sp[0].d_states.as<uint32_t>(), b->sp[1].d_states.as<uint32_t>(), b->sp[0].dim,
                           b->sp[1].dim, static_cast<const double *>(psi), red);
    else if (dtype == HPHI_C64)
        hipLaunchKernelGGL(k_docc_hub<float>, dim3(grid_for(b->dim, 4)), dim3(kBlock), 0, st,
                           b->sp[0].d_states.as<uint32_t>(), b->sp[1].d_states.as<uint32_t>(), b->sp[0].dim,
                           b->sp[1].dim, static_cast<const float *>(psi), red);
    else
        return fail(HPHI_ERR_INVALID_ARG, "double occupancy takes a complex vector");
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_trace(hphi_ham *h, Reduce red, hipStream_t st)
{
    const hphi_basis *b = h->basis;
    if (h->kind == 2) return launch_gc_trace(h, red, st);
    if (h->kind == 3) return launch_spin_s_trace(h, red, st);
    if (h->kind == 0) {
        if (!b->sp[0].materialized() || b->sp[0].state_bytes != 4)
            return fail(HPHI_ERR_UNSUPPORTED, "trace needs a materialized basis with N <= 32");
        hipLaunchKernelGGL(k_trace_spin, dim3(grid_for(b->dim, 4)), dim3(kBlock), 0, st,
                           b->sp[0].d_states.as<uint32_t>(), b->dim, h->d_bonds.as<SpinBondDev>(),
                           h->n_bonds, h->has_field ? h->d_hz.as<double>() : nullptr, b->n_sites, red);
    } else {
        hipLaunchKernelGGL(k_trace_hub, dim3(grid_for(b->dim, 4)), dim3(kBlock), 0, st,
                           b->sp[0].d_states.as<uint32_t>(), b->sp[1].d_states.as<uint32_t>(),
                           b->sp[0].dim, b->sp[1].dim, h->hub.u_site.as<double>(), h->hub.pairs.as<HubPairDev>(),
                           h->hub.n_pairs, red);
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// ------------------------------------------------------------- S^z(q) --
// b[x] = (sum_l phase_l S^z_l(x)) psi[x], S^z_l = +-1/2 by bit l.
__global__ void k_szq(const uint32_t *states, int64_t dim, int n_sites, const double *phase,
                      const double *psi, double *b)
{
    __shared__ double ph[128];
    for (int i = threadIdx.x; i < 2 * n_sites; i += blockDim.x) ph[i] = phase[i];
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = states[r];
        double re = 0.0, im = 0.0;
        for (int l = 0; l < n_sites; ++l) {
            const double sz = ((x >> l) & 1u) ? 0.5 : -0.5;
            re += sz * ph[2 * l];
            im += sz * ph[2 * l + 1];
        }
        const double p = psi[r];
        b[2 * r] = re * p;
        b[2 * r + 1] = im * p;
    }
}

// Hubbard basis: S^z_l = (n_l,up - n_l,dn) / 2; index r = r_up * dim_dn + r_dn.
// One up row per block iteration, the threads over the down states.
__global__ void k_szq_hub(const uint32_t *ups, const uint32_t *dns, int64_t dim_up, int64_t dim_dn,
                          int n_sites, const double *phase, const double *psi, double *b)
{
    __shared__ double ph[128];
    for (int i = threadIdx.x; i < 2 * n_sites; i += blockDim.x) ph[i] = phase[i];
    __syncthreads();
    for (int64_t ru = blockIdx.x; ru < dim_up; ru += gridDim.x) {
        const uint32_t x = ups[ru];
        for (int64_t rd = threadIdx.x; rd < dim_dn; rd += blockDim.x) {
            const uint32_t y = dns[rd];
            double re = 0.0, im = 0.0;
            for (int l = 0; l < n_sites; ++l) {
                const double sz = 0.5 * ((double)((x >> l) & 1u) - (double)((y >> l) & 1u));
                re += sz * ph[2 * l];
                im += sz * ph[2 * l + 1];
            }
            const int64_t r = ru * dim_dn + rd;
            const double p = psi[r];
            b[2 * r] = re * p;
            b[2 * r + 1] = im * p;
        }
    }
}

int launch_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st)
{
    const hphi_basis *bs = h->basis;
    if (bs->dim == 0) return HPHI_OK;
    if (h->kind == 2) return launch_gc_szq(h, phase_dev, psi, b, st);
    if (h->kind == 3) return launch_spin_s_szq(h, phase_dev, psi, b, st);
    if (h->kind == 0) {
        if (!bs->sp[0].materialized() || bs->sp[0].state_bytes != 4)
            return fail(HPHI_ERR_UNSUPPORTED, "S^z(q) needs a stored spin basis with N <= 32");
        hipLaunchKernelGGL(k_szq, dim3(grid_for(bs->dim, 2)), dim3(kBlock), 0, st,
                           bs->sp[0].d_states.as<uint32_t>(), bs->dim, bs->n_sites, phase_dev,
                           (const double *)psi, (double *)b);
    } else {
        const int64_t du = bs->sp[0].dim, dd = bs->sp[1].dim;
        const unsigned grid = (unsigned)std::min<int64_t>(du, 65536);
        hipLaunchKernelGGL(k_szq_hub, dim3(grid), dim3(kBlock), 0, st,
                           bs->sp[0].d_states.as<uint32_t>(), bs->sp[1].d_states.as<uint32_t>(), du, dd,
                           bs->n_sites, phase_dev, (const double *)psi, (double *)b);
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

namespace hphi {

// dst[k * row + i] = src[i] (i < n), k = counter[which], then counter[which]
// advances: results of successive steps land in successive rows of a device
// staging array, with the same launch for every step (graph replay).
__global__ void k_record(const double *src, int n, double *dst, int row, int *counter, int which)
{
    const int k = counter[which];
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[(size_t)k * row + i] = src[i];
    __syncthreads();
    if (threadIdx.x == 0) counter[which] = k + 1;
}

int launch_record(const double *src, int n, double *dst, int row, int *counter, int which, hipStream_t st)
{
    hipLaunchKernelGGL(k_record, dim3(1), dim3(64), 0, st, src, n, dst, row, counter, which);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

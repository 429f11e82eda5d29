// Block kernels of the LOBPCG eigensolver (HPhi update paper Sec. 3.3). A
// block is an array of separate FP64 vectors (device pointer arrays), so
// every H*v of the solver is an ordinary launch of any model's kernel.
//   k_diag_*   : H_xx per state (the point-Jacobi preconditioner's diagonal)
//   k_gram     : G = X^T Y for blocks of a <= 32 and b <= 32 vectors, FP64,
//                per-block partials summed in block order (run-to-run
//                identical)
//   k_lincomb  : out_n = sum_m C[m][n] V_m (C in LDS)
//   k_resid    : r_n = HPhi_n - E_n Phi_n, |r_n|^2, then optionally
//                r_n /= (H_xx - E_shift); E_n read from a Gram diagonal
//   k_scale    : x_n *= 1 / sqrt(G_nn), G a Gram matrix on the device
#include "kern_common.h"
#include "hub_pairs.h"

namespace hphi {

constexpr int kGramMax = 32;

// Last workgroup of a launch: result[t] = sum over blocks of
// partial[b * nres + t], one wave per result, lanes over blocks in a fixed
// stride and a fixed shuffle tree (run-to-run identical).
__device__ __forceinline__ void finish_waves(const double *partial, unsigned nblocks, int nres, double *result)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int t = wid; t < nres; t += nw) {
        double s = 0.0;
        for (unsigned b = lane; b < nblocks; b += 64) s += __builtin_nontemporal_load(&partial[(size_t)b * nres + t]);
        s = wave_sum(s);
        if (lane == 0) result[t] = s;
    }
}

__global__ __launch_bounds__(kBlock) void k_diag_spin(const uint32_t *states, int64_t dim, const SpinBondDev *bonds,
                                                      int nb, const double *hz, int n_sites, double *out)
{
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
        out[r] = d;
    }
}

__global__ __launch_bounds__(kBlock) void k_diag_hub(const uint32_t *ups, const uint32_t *dns, int64_t dup,
                                                     int64_t ddn, const double *u_site, const HubPairDev *pairs,
                                                     int np, double *out)
{
    const int64_t n = dup * ddn;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
         t += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t u = ups[t / ddn], dn = dns[t % ddn];
        uint32_t both = u & dn;
        double d = 0.0;
        while (both) {
            d += u_site[__builtin_ctz(both)];
            both &= both - 1u;
        }
        if (np) d += hub_pair_diag(pairs, np, u, dn);
        out[t] = d;
    }
}

// Thread (row group rr, lane i): AP lanes per row (AP >= a, a power of two),
// 256 / AP rows per pass; b accumulators per thread.
template <int AP>
__global__ __launch_bounds__(kBlock) void k_gram(const double *const *X, int a, const double *const *Y, int b,
                                                 int64_t dim, double *partial, unsigned *counter, double *result)
{
    constexpr int RPB = kBlock / AP;
    __shared__ double sw[kBlock / kWave][AP][kGramMax];
    __shared__ unsigned s_last;
    const int i = threadIdx.x % AP, rr = threadIdx.x / AP;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double acc[kGramMax];
#pragma unroll
    for (int j = 0; j < kGramMax; ++j) acc[j] = 0.0;
    if (i < a) {
        const double *xi = X[i];
        for (int64_t r = (int64_t)blockIdx.x * RPB + rr; r < dim; r += (int64_t)gridDim.x * RPB) {
            const double xv = xi[r];
#pragma unroll
            for (int j = 0; j < kGramMax; ++j)
                if (j < b) acc[j] += xv * Y[j][r];
        }
    }
    // rows of one wave with the same lane i, then waves
#pragma unroll
    for (int j = 0; j < kGramMax; ++j)
        for (int off = 32; off >= AP; off >>= 1) acc[j] += __shfl_xor(acc[j], off, kWave);
    if (lane < AP)
#pragma unroll
        for (int j = 0; j < kGramMax; ++j) sw[wid][lane][j] = acc[j];
    __syncthreads();
    const int nres = a * b;
    for (int t = threadIdx.x; t < nres; t += blockDim.x) {
        const int ii = t / b, jj = t % b;
        double s = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) s += sw[w][ii][jj];
        partial[(size_t)blockIdx.x * nres + t] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finish_waves(partial, gridDim.x, nres, result);
    __syncthreads();
    if (threadIdx.x == 0) {
        *counter = 0u;
        __threadfence();
    }
}

// Small blocks (a, b <= 8): one thread per row holds all a * b products, so
// every load of a wave is a contiguous run of rows.
__global__ __launch_bounds__(kBlock) void k_gram8(const double *const *X, int a, const double *const *Y, int b,
                                                  int64_t dim, double *partial, unsigned *counter, double *result)
{
    __shared__ double sw[kBlock / kWave][64];
    __shared__ unsigned s_last;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    double acc[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[i][j] = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        double x[8], y[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i] = i < a ? X[i][r] : 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) y[j] = j < b ? Y[j][r] : 0.0;
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[i][j] += x[i] * y[j];
    }
    const int nres = a * b;
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if (i < a && j < b) {
                const double v = wave_sum(acc[i][j]);
                if (lane == 0) sw[wid][i * b + j] = v;
            }
        }
    __syncthreads();
    for (int t = threadIdx.x; t < nres; t += blockDim.x) {
        double sm = 0.0;
        for (int w = 0; w < kBlock / kWave; ++w) sm += sw[w][t];
        partial[(size_t)blockIdx.x * nres + t] = sm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finish_waves(partial, gridDim.x, nres, result);
    __syncthreads();
    if (threadIdx.x == 0) {
        *counter = 0u;
        __threadfence();
    }
}

// out_n[r] = sum_m C[m * nout + n] V_m[r]; nin <= 96, nout <= 32.
__global__ __launch_bounds__(kBlock) void k_lincomb(const double *const *V, int nin, const double *C, double *const *out,
                                                    int nout, int64_t dim)
{
    __shared__ double sc[96 * kGramMax];
    for (int t = threadIdx.x; t < nin * nout; t += blockDim.x) sc[t] = C[t];
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        double acc[kGramMax];
#pragma unroll
        for (int n = 0; n < kGramMax; ++n) acc[n] = 0.0;
        for (int m = 0; m < nin; ++m) {
            const double x = V[m][r];
#pragma unroll
            for (int n = 0; n < kGramMax; ++n)
                if (n < nout) acc[n] += sc[m * nout + n] * x;
        }
#pragma unroll
        for (int n = 0; n < kGramMax; ++n)
            if (n < nout) out[n][r] = acc[n];
    }
}

// r_n = HPhi_n - E_n Phi_n (E_n = E[n * estride]); partial |r_n|^2 per
// block; then with a diagonal r_n /= (d - shift).
__global__ __launch_bounds__(kBlock) void k_resid(const double *const *HPhi, const double *const *Phi,
                                                  double *const *R, int m, const double *E, int estride,
                                                  const double *d, double shift, int64_t dim, double *partial,
                                                  unsigned *counter, double *result)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[kGramMax];
    __shared__ unsigned s_last;
    for (int n = 0; n < m; ++n) {
        const double e = E[n * estride];
        const double sft = shift;
        double acc = 0.0;
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
             r += (int64_t)gridDim.x * blockDim.x) {
            double x = HPhi[n][r] - e * Phi[n][r];
            acc += x * x;
            if (d) x /= (d[r] - sft);
            R[n][r] = x;
        }
        double v[1] = {acc};
        block_sum<1>(v, sh);
        if (threadIdx.x == 0) blk[n] = v[0];
    }
    __syncthreads();
    if (threadIdx.x < m) partial[(size_t)blockIdx.x * m + threadIdx.x] = blk[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = (atomicAdd(counter, 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    finish_waves(partial, gridDim.x, m, result);
    __syncthreads();
    if (threadIdx.x == 0) {
        *counter = 0u;
        __threadfence();
    }
}

// x_n *= 1 / sqrt(g[n * (ld + 1)]) (0 when that diagonal entry is not positive)
__global__ __launch_bounds__(kBlock) void k_scale(double *const *X, int m, const double *g, int ld, int64_t dim)
{
    for (int n = 0; n < m; ++n) {
        const double gn = g[(size_t)n * (ld + 1)];
        const double f = gn > 0.0 ? 1.0 / sqrt(gn) : 0.0;
        for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
             r += (int64_t)gridDim.x * blockDim.x)
            X[n][r] *= f;
    }
}

static int lob_grid(int64_t n)
{
    int64_t g = (n + kBlock - 1) / kBlock;
    if (g > 1024) g = 1024;
    if (g < 1) g = 1;
    return (int)g;
}

int launch_diag(hphi_ham *h, double *out, hipStream_t st)
{
    const hphi_basis *b = h->basis;
    if (h->kind == 2) return launch_gc_diag(h, out, st);
    if (h->kind == 3) return launch_spin_s_diag(h, out, st);
    if (h->kind == 0) {
        if (!b->sp[0].materialized() || b->sp[0].state_bytes != 4)
            return fail(HPHI_ERR_UNSUPPORTED, "the diagonal needs a stored basis (N <= 32)");
        hipLaunchKernelGGL(k_diag_spin, dim3(lob_grid(b->dim)), dim3(kBlock), 0, st, b->sp[0].d_states.as<uint32_t>(),
                           b->dim, h->d_bonds.as<SpinBondDev>(), h->n_bonds,
                           h->has_field ? h->d_hz.as<double>() : nullptr, b->n_sites, out);
    } else {
        hipLaunchKernelGGL(k_diag_hub, dim3(lob_grid(b->dim)), dim3(kBlock), 0, st, b->sp[0].d_states.as<uint32_t>(),
                           b->sp[1].d_states.as<uint32_t>(), b->sp[0].dim, b->sp[1].dim,
                           h->hub.u_site.as<double>(), h->hub.pairs.as<HubPairDev>(), h->hub.n_pairs, out);
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_gram(const double *const *X, int a, const double *const *Y, int b, int64_t dim, Reduce red,
                hipStream_t st)
{
    if (a < 1 || a > kGramMax || b < 1 || b > kGramMax) return fail(HPHI_ERR_INVALID_ARG, "gram %d x %d", a, b);
    int g = lob_grid(dim / 4 + 1);
    if ((int64_t)g * a * b > kReduceSlots) g = (int)(kReduceSlots / (a * b));
    if (a <= 8 && b <= 8) hipLaunchKernelGGL(k_gram8, dim3(g), dim3(kBlock), 0, st, X, a, Y, b, dim, red.partial, red.counter, red.result);
    else if (a <= 8) hipLaunchKernelGGL(k_gram<8>, dim3(g), dim3(kBlock), 0, st, X, a, Y, b, dim, red.partial, red.counter, red.result);
    else if (a <= 16) hipLaunchKernelGGL(k_gram<16>, dim3(g), dim3(kBlock), 0, st, X, a, Y, b, dim, red.partial, red.counter, red.result);
    else hipLaunchKernelGGL(k_gram<32>, dim3(g), dim3(kBlock), 0, st, X, a, Y, b, dim, red.partial, red.counter, red.result);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_lincomb(const double *const *V, int nin, const double *C, double *const *out, int nout, int64_t dim,
                   hipStream_t st)
{
    if (nin < 1 || nin > 96 || nout < 1 || nout > kGramMax)
        return fail(HPHI_ERR_INVALID_ARG, "lincomb %d -> %d", nin, nout);
    hipLaunchKernelGGL(k_lincomb, dim3(lob_grid(dim)), dim3(kBlock), 0, st, V, nin, C, out, nout, dim);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_resid(const double *const *HPhi, const double *const *Phi, double *const *R, int m, const double *E,
                 int estride, const double *d, double shift, int64_t dim, Reduce red, hipStream_t st)
{
    if (m < 1 || m > kGramMax) return fail(HPHI_ERR_INVALID_ARG, "resid block %d", m);
    hipLaunchKernelGGL(k_resid, dim3(lob_grid(dim)), dim3(kBlock), 0, st, HPhi, Phi, R, m, E, estride, d, shift,
                       dim, red.partial, red.counter, red.result);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_scale_block(double *const *X, int m, const double *g, int ld, int64_t dim, hipStream_t st)
{
    hipLaunchKernelGGL(k_scale, dim3(lob_grid(dim)), dim3(kBlock), 0, st, X, m, g, ld, dim);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

// Batched small-sector Lanczos: one workgroup runs a whole solve.
//
// For sectors of up to a few hundred thousand states an H*v takes a few
// microseconds, so a solve driven by one kernel launch per step is bound by
// launch latency. Here a launch carries many independent requests (each its
// own spin Hamiltonian, sector, iteration count and seed); workgroup b runs
// the complete recurrence of request b (the plain Lanczos of the HPhi update
// paper's introduction, without reorthogonalization):
//   q_0 = r (SplitMix64 uniform [-1/2, 1/2), the same stream as the
//   single-solve path), s_0 = 1/|q_0|;
//   w = s_k H q_k - beta_k s_{k-1} q_{k-1};  alpha_k = s_k <q_k, w>;
//   w -= alpha_k s_k q_k;  beta_{k+1} = |w|;  q_{k+1} = w, s_{k+1} = 1/beta_{k+1};
// with FP64 block reductions in a fixed order, so a request's result does
// not depend on which other requests share the launch. The vectors live in
// global memory (L2-resident at these sizes); the rank tables are staged in
// LDS when they fit.
#include "kern_common.h"

namespace hphi {

typedef const __attribute__((address_space(4))) SpinBondDev CSpinBond;
typedef const __attribute__((address_space(4))) double CDouble;

struct BatchItemDev {
    const uint32_t *states;
    int64_t dim;
    const SpinBondDev *bonds;
    int nb;
    int n_lo, n_hi;
    const uint32_t *lo_rank;
    const uint32_t *hi_off;
    const double *hz;
    int n_sites;
    int iters;
    uint64_t seed;
    double *q;          // 3 * dim workspace
    double *alpha;      // iters
    double *beta;       // iters + 1
    int *done;          // [0] steps done, [1] breakdown flag
};

constexpr int kBatchThreads = 256;
constexpr int kBatchLdsTab = 8192;   // uint32 entries of staged tables

__device__ __forceinline__ double batch_sum(double x, double *sh)
{
    double v[1] = {x};
    block_sum<1>(v, sh);
    __shared__ double bcast;
    if (threadIdx.x == 0) bcast = v[0];
    __syncthreads();
    const double r = bcast;
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kBatchThreads) void k_lanczos_batch(const BatchItemDev *items)
{
    __shared__ double sh[kBatchThreads / kWave];
    __shared__ uint32_t s_tab[kBatchLdsTab];
    const BatchItemDev it = items[blockIdx.x];
    // uniform tables through the scalar cache (the item is read from memory,
    // so without the cast every lane would load them with vector loads)
    const CSpinBond *bc = (const CSpinBond *)(it.bonds);
    const CDouble *hzc = (const CDouble *)(it.hz);
    const int64_t dim = it.dim;
    const uint32_t lomask = (1u << it.n_lo) - 1u;
    const uint32_t nl = 1u << it.n_lo, nh = 1u << it.n_hi;
    const uint32_t *lo = it.lo_rank, *hi = it.hi_off;
    if (nl + nh <= (uint32_t)kBatchLdsTab) {
        for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) s_tab[i] = it.lo_rank[i];
        for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) s_tab[nl + i] = it.hi_off[i];
        lo = s_tab;
        hi = s_tab + nl;
    }
    double *q[3] = {it.q, it.q + dim, it.q + 2 * dim};
    // start vector and its norm
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
        const double x = u53(splitmix64_at(it.seed, (uint64_t)r)) - 0.5;
        q[0][r] = x;
        acc += x * x;
    }
    const double n0 = batch_sum(acc, sh);
    double s_cur = 1.0 / sqrt(n0), s_prev = 0.0, b_cur = 0.0;
    int cur = 0, prev = 2, wb = 1, k = 0, brk = 0;
    for (; k < it.iters; ++k) {
        const double c1 = s_cur, c2 = -b_cur * s_prev;
        const double *qc = q[cur], *qp = q[prev];
        double *w = q[wb];
        double pa = 0.0;
        for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
            const uint32_t x = it.states[r];
            double hv = 0.0, diag = 0.0;
            for (int b = 0; b < it.nb; ++b) {
                const uint32_t m = (uint32_t)bc[b].mask, t = x & m;
                if (t == 0u || t == m) {
                    diag += bc[b].jz4;
                } else {
                    diag -= bc[b].jz4;
                    const uint32_t y = x ^ m;
                    hv += bc[b].jxy2 * qc[hi[y >> it.n_lo] + lo[y & lomask]];
                }
            }
            if (it.hz)
                for (int i = 0; i < it.n_sites; ++i) diag -= hzc[i] * (((x >> i) & 1u) ? 0.5 : -0.5);
            double o = c1 * (hv + diag * qc[r]);
            if (k > 0) o += c2 * qp[r];
            w[r] = o;
            pa += qc[r] * o;
        }
        const double al = s_cur * batch_sum(pa, sh);
        const double f = al * s_cur;
        double pb = 0.0;
        for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
            const double x = w[r] - f * qc[r];
            w[r] = x;
            pb += x * x;
        }
        const double bn = sqrt(batch_sum(pb, sh));
        if (threadIdx.x == 0) {
            it.alpha[k] = al;
            it.beta[k + 1] = bn;
        }
        if (!(bn > 1e-13 * fmax(1.0, fabs(al)))) {
            brk = 1;
            ++k;
            break;
        }
        s_prev = s_cur;
        s_cur = 1.0 / bn;
        b_cur = bn;
        const int op = prev;
        prev = cur;
        cur = wb;
        wb = op;
    }
    if (threadIdx.x == 0) {
        it.done[0] = k;
        it.done[1] = brk;
        it.beta[0] = 0.0;
    }
}

// LDS-resident variant for sectors whose vector fits next to the rank
// tables in LDS: q_k lives in LDS (the H*v gathers read it there), q_{k-1}
// and w in global memory. The update step moves q_k to the q_{k-1} buffer
// and writes q_{k+1} into LDS row by row (each thread touches only its own
// rows), so a step is one gather pass from LDS plus four streaming passes.
constexpr int kBatchLdsThreads = 1024;

__global__ __launch_bounds__(kBatchLdsThreads) void k_lanczos_batch_lds(const BatchItemDev *items)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ double sh[kBatchLdsThreads / kWave];
    const BatchItemDev it = items[blockIdx.x];
    // uniform tables through the scalar cache (the item is read from memory,
    // so without the cast every lane would load them with vector loads)
    const CSpinBond *bc = (const CSpinBond *)(it.bonds);
    const CDouble *hzc = (const CDouble *)(it.hz);
    const int64_t dim = it.dim;
    double *Q = reinterpret_cast<double *>(smem_raw);
    uint32_t *lo = reinterpret_cast<uint32_t *>(Q + dim);
    const uint32_t nl = 1u << it.n_lo, nh = 1u << it.n_hi;
    uint32_t *hi = lo + nl;
    for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) lo[i] = it.lo_rank[i];
    for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) hi[i] = it.hi_off[i];
    const uint32_t lomask = nl - 1u;
    double *P = it.q, *Wv = it.q + dim;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
        const double x = u53(splitmix64_at(it.seed, (uint64_t)r)) - 0.5;
        Q[r] = x;
        acc += x * x;
    }
    const double n0 = batch_sum(acc, sh);
    double s_cur = 1.0 / sqrt(n0), s_prev = 0.0, b_cur = 0.0;
    int k = 0, brk = 0;
    for (; k < it.iters; ++k) {
        const double c1 = s_cur, c2 = -b_cur * s_prev;
        double pa = 0.0;
        for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
            const uint32_t x = it.states[r];
            double hv = 0.0, diag = 0.0;
            for (int b = 0; b < it.nb; ++b) {
                const uint32_t m = (uint32_t)bc[b].mask, t = x & m;
                if (t == 0u || t == m) {
                    diag += bc[b].jz4;
                } else {
                    diag -= bc[b].jz4;
                    const uint32_t y = x ^ m;
                    hv += bc[b].jxy2 * Q[hi[y >> it.n_lo] + lo[y & lomask]];
                }
            }
            if (it.hz)
                for (int i = 0; i < it.n_sites; ++i) diag -= hzc[i] * (((x >> i) & 1u) ? 0.5 : -0.5);
            const double qr = Q[r];
            double o = c1 * (hv + diag * qr);
            if (k > 0) o += c2 * P[r];
            Wv[r] = o;
            pa += qr * o;
        }
        const double al = s_cur * batch_sum(pa, sh);
        const double f = al * s_cur;
        double pb = 0.0;
        for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
            const double qr = Q[r];
            const double x = Wv[r] - f * qr;
            P[r] = qr;
            Q[r] = x;
            pb += x * x;
        }
        const double bn = sqrt(batch_sum(pb, sh));
        if (threadIdx.x == 0) {
            it.alpha[k] = al;
            it.beta[k + 1] = bn;
        }
        if (!(bn > 1e-13 * fmax(1.0, fabs(al)))) {
            brk = 1;
            ++k;
            break;
        }
        s_prev = s_cur;
        s_cur = 1.0 / bn;
        b_cur = bn;
    }
    if (threadIdx.x == 0) {
        it.done[0] = k;
        it.done[1] = brk;
        it.beta[0] = 0.0;
    }
}

size_t batch_lds_bytes(int64_t dim, int n_lo, int n_hi)
{
    return sizeof(double) * (size_t)dim + sizeof(uint32_t) * ((size_t(1) << n_lo) + (size_t(1) << n_hi));
}

int launch_lanczos_batch(const void *items_dev, int n, hipStream_t st, size_t lds_bytes)
{
    if (lds_bytes > 0) {
        hipFuncSetAttribute((const void *)k_lanczos_batch_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
        hipLaunchKernelGGL(k_lanczos_batch_lds, dim3(n), dim3(kBatchLdsThreads), lds_bytes, st,
                           (const BatchItemDev *)items_dev);
    } else {
        hipLaunchKernelGGL(k_lanczos_batch, dim3(n), dim3(kBatchThreads), 0, st, (const BatchItemDev *)items_dev);
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

size_t batch_item_size() { return sizeof(BatchItemDev); }

int fill_batch_item(hphi_ham *h, int iters, uint64_t seed, double *q, double *alpha, double *beta, int *done,
                    void *out)
{
    const hphi_basis *b = h->basis;
    const Species &s = b->sp[0];
    if (h->kind != 0 || !s.materialized() || s.state_bytes != 4 || !s.d_hi_off32.p)
        return fail(HPHI_ERR_UNSUPPORTED, "batched Lanczos takes spin Hamiltonians with a stored basis");
    BatchItemDev d{};
    d.states = s.d_states.as<uint32_t>();
    d.dim = s.dim;
    d.bonds = h->d_bonds.as<SpinBondDev>();
    d.nb = h->n_bonds;
    d.n_lo = s.n_lo;
    d.n_hi = s.n_hi;
    d.lo_rank = s.d_lo_rank.as<uint32_t>();
    d.hi_off = s.d_hi_off32.as<uint32_t>();
    d.hz = h->has_field ? h->d_hz.as<double>() : nullptr;
    d.n_sites = b->n_sites;
    d.iters = iters;
    d.seed = seed;
    d.q = q;
    d.alpha = alpha;
    d.beta = beta;
    d.done = done;
    *static_cast<BatchItemDev *>(out) = d;
    return HPHI_OK;
}

} // namespace hphi

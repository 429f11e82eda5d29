// Spin-1/2 H*v on the full 2^N space (SpinGC keyword of the HPhi update
// paper, Sec. 4.1; the XYZ bonds and fields of its spin models):
//   H = sum_b [jx S^x_i S^x_j + jy S^y_i S^y_j + jz S^z_i S^z_j]
//       - sum_i (hx_i S^x_i + hz_i S^z_i).
// The index of a state is its configuration, so every off-diagonal term is
// a bit flip x -> x ^ M (M = {i, j} for a bond, {i} for a transverse field)
// with a coefficient that depends only on whether bits i and j agree:
// (jx - jy)/4 when they do, (jx + jy)/4 when they do not, -hx/2 for a field.
//
// Bit windows. A gather x ^ M with a high bit in M jumps 2^bit states, so
// a plain per-state kernel streams one far block of v per high term. Here a
// pass takes one window of bits: its tiles are the 2^(lowb + q) states that
// vary in the low bits (16 consecutive states: whole 128-byte lines) and the
// q window bits, with every other bit fixed by the tile index. A tile is
// staged in LDS once and every term whose flip mask lies in the window is
// applied from there. The host plans windows so that every term falls in
// one; each pass reads v and the partial w and writes w once (the first
// pass adds the diagonal and writes w without reading it; the last applies
// the caller's epilogue and the FP64 dot products).
#include "kern_common.h"
#include "row_finish.h"

namespace hphi {

struct GcKArgs {
    int lowb, q;
    uint32_t compmask;        // bits fixed per tile (scattered from the tile index)
    int64_t ntiles;
    const uint32_t *offw;     // 2^q: window index -> window bits
    const GcTermDev *terms;
    int nterms;
    const GcDiagDev *diag;    // first pass: S^z S^z bonds
    int ndiag;
    const double *hz;         // first pass: longitudinal fields (or null)
    int n_sites;
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    void *raw_out;
    const double *coef;
    int coef_cplx;
    int nd;
    int dot_raw;
    Reduce red;
};

// The bits of t placed, in order, on the set bits of mask.
__device__ __forceinline__ uint64_t scatter_bits(uint64_t t, uint32_t mask)
{
    uint64_t out = 0;
    while (mask) {
        const int b = __builtin_ctz(mask);
        out |= (t & 1ull) << b;
        t >>= 1;
        mask &= mask - 1u;
    }
    return out;
}

template <typename S, int NV, bool FIRST, bool LAST, bool DOTS>
__global__ __launch_bounds__(1024) void k_spin_gc(GcKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int L = 1 << (a.lowb + a.q);
    // LDS: the tile, the window's term records and S^z S^z bonds (read with
    // wave-uniform addresses: broadcasts), the window-bit scatter table
    S *s_v = reinterpret_cast<S *>(smem_raw);
    GcTermDev *s_terms = reinterpret_cast<GcTermDev *>(s_v + (size_t)L * NV);
    GcDiagDev *s_diag = reinterpret_cast<GcDiagDev *>(s_terms + a.nterms);
    uint32_t *s_offw = reinterpret_cast<uint32_t *>(s_diag + (FIRST ? a.ndiag : 0));
    __shared__ double sh_red[2 * NV * 16];
    __shared__ double sh_blk[2 * NV];
    const int tid = threadIdx.x, T = blockDim.x;
    for (int k = tid; k < (1 << a.q); k += T) s_offw[k] = a.offw[k];
    for (int k = tid; k < a.nterms; k += T) s_terms[k] = a.terms[k];
    if constexpr (FIRST)
        for (int k = tid; k < a.ndiag; k += T) s_diag[k] = a.diag[k];
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *w = static_cast<S *>(a.w);   // also written through the epilogue's pointer
    const uint32_t lowmask = (1u << a.lowb) - 1u;
    const EpiArgs<S> ep{w, static_cast<const S *>(a.u), static_cast<S *>(a.acc_out), static_cast<S *>(a.raw_out),
                        a.coef, a.coef_cplx, a.dot_raw};
    RowFinish<S, NV, DOTS> fin;
    fin.init(ep);

    for (int64_t t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
        const uint64_t base = scatter_bits((uint64_t)t, a.compmask);
        __syncthreads();   // s_offw loaded; the previous tile is no longer read
        for (int l = tid; l < L; l += T) {
            const uint64_t x = base | s_offw[l >> a.lowb] | (uint32_t)(l & lowmask);
#pragma unroll
            for (int j = 0; j < NV; ++j) s_v[(size_t)l * NV + j] = v[x * NV + j];
        }
        __syncthreads();
        for (int l = tid; l < L; l += T) {
            const uint64_t x = base | s_offw[l >> a.lowb] | (uint32_t)(l & lowmask);
            S hv[NV];
            if constexpr (FIRST) {
                S dg = (S)0;
#pragma unroll 4
                for (int b = 0; b < a.ndiag; ++b) {
                    const GcDiagDev dd = s_diag[b];
                    const uint32_t tb = (uint32_t)x & dd.mask;
                    dg += (tb == 0u || tb == dd.mask) ? (S)dd.jz4 : (S)-dd.jz4;
                }
                if (a.hz)
                    for (int i = 0; i < a.n_sites; ++i) dg -= (S)a.hz[i] * (((x >> i) & 1ull) ? (S)0.5 : (S)-0.5);
#pragma unroll
                for (int j = 0; j < NV; ++j) hv[j] = dg * s_v[(size_t)l * NV + j];
            } else {
#pragma unroll
                for (int j = 0; j < NV; ++j) hv[j] = (S)0;
            }
#pragma unroll 4
            for (int k = 0; k < a.nterms; ++k) {
                const GcTermDev tm = s_terms[k];
                const int p = l ^ (int)tm.mloc;
                const bool par = (((uint32_t)l >> tm.pi) ^ ((uint32_t)l >> tm.pj)) & 1u ? false : true;
                const S c = par ? (S)tm.cpar : (S)tm.canti;
#pragma unroll
                for (int j = 0; j < NV; ++j) hv[j] += c * s_v[(size_t)p * NV + j];
            }
            if constexpr (!FIRST) {
#pragma unroll
                for (int j = 0; j < NV; ++j) hv[j] += w[x * NV + j];
            }
            if constexpr (!LAST) {
#pragma unroll
                for (int j = 0; j < NV; ++j) w[x * NV + j] = hv[j];
            } else {
                S me[NV];
#pragma unroll
                for (int j = 0; j < NV; ++j) me[j] = s_v[(size_t)l * NV + j];
                fin.apply(hv, me, (size_t)x, ep);
            }
        }
    }
    fin.reduce(a.red, sh_red, sh_blk);
}

template <typename S, int NV, bool FIRST, bool LAST>
static void launch_gc_pass(const GcKArgs &a, int grid, size_t lds, hipStream_t st)
{
    auto go = [&](auto kern) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, a);
    };
    if (LAST && a.nd) go(k_spin_gc<S, NV, FIRST, LAST, LAST>);
    else go(k_spin_gc<S, NV, FIRST, LAST, false>);
}

template <typename S, int NV>
static int launch_gc_t(hphi_ham *h, const MultArgs &m)
{
    const int esz = NV * (int)sizeof(S);
    const int pidx = esz == 4 ? 0 : (esz == 8 ? 1 : 2);
    HPHI_TRY(gc_plan_build(h, pidx));
    const GcPlan &plan = h->gc_plan[pidx];
    const hphi_basis *b = h->basis;
    const int nw = (int)plan.wins.size();
    // later passes read v, u and the partial w: none may alias w
    if (nw > 1 && (m.v == m.w || (m.u && m.u == m.w) || (m.acc && m.acc == m.w)))
        return fail(HPHI_ERR_INVALID_ARG, "SpinGC H*v: w may not alias v, u or acc");
    GcKArgs a{};
    a.lowb = plan.lowb;
    a.diag = h->gc_diag.as<GcDiagDev>();
    a.ndiag = h->gc_ndiag;
    a.hz = h->gc_has_hz ? h->gc_hz.as<double>() : nullptr;
    a.n_sites = b->n_sites;
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.raw_out = m.raw_out;
    a.coef = m.coef;
    a.coef_cplx = m.coef_cplx;
    a.nd = m.dots;
    a.dot_raw = m.dot_raw;
    a.red = m.red;
    const int ncu = b->ctx->n_cu > 0 ? b->ctx->n_cu : 256;
    for (int k = 0; k < nw; ++k) {
        const GcWindow &wn = plan.wins[k];
        a.q = wn.q;
        a.compmask = wn.compmask;
        a.ntiles = (int64_t)1 << (b->n_sites - plan.lowb - wn.q);
        a.offw = plan.offw.as<uint32_t>() + wn.offw_first;
        a.terms = plan.terms.as<GcTermDev>() + wn.term_first;
        a.nterms = wn.term_count;
        const size_t lds = ((size_t)1 << (plan.lowb + wn.q)) * NV * sizeof(S) + sizeof(GcTermDev) * wn.term_count +
                           (k == 0 ? sizeof(GcDiagDev) * (size_t)a.ndiag : 0) + ((size_t)1 << wn.q) * 4;
        if (lds > 160 * 1024) return fail(HPHI_ERR_UNSUPPORTED, "SpinGC window tile and terms beyond the LDS");
        const int grid = (int)std::min<int64_t>(a.ntiles, 2 * (int64_t)ncu);
        if (a.nd && (int64_t)grid * 2 * NV > kReduceSlots)
            return fail(HPHI_ERR_UNSUPPORTED, "SpinGC grid beyond the reduction scratch");
        const bool first = k == 0, last = k == nw - 1;
        if (first && last) launch_gc_pass<S, NV, true, true>(a, grid, lds, m.stream);
        else if (first) launch_gc_pass<S, NV, true, false>(a, grid, lds, m.stream);
        else if (last) launch_gc_pass<S, NV, false, true>(a, grid, lds, m.stream);
        else launch_gc_pass<S, NV, false, false>(a, grid, lds, m.stream);
        HPHI_HIP(hipGetLastError());
    }
    return HPHI_OK;
}

int launch_gc_mult(hphi_ham *h, const MultArgs &m)
{
    if (m.lz || m.lz_q) return fail(HPHI_ERR_UNSUPPORTED, "SpinGC: no fused Lanczos update");
    if (m.ld > 0 && m.ld != h->basis->dim) return fail(HPHI_ERR_UNSUPPORTED, "SpinGC: no row pitch");
    const int nv = m.nvec * dtype_lanes(m.dtype);
    const bool f32 = dtype_is_f32(m.dtype);
    if (nv == 1) return f32 ? launch_gc_t<float, 1>(h, m) : launch_gc_t<double, 1>(h, m);
    if (nv == 2) return f32 ? launch_gc_t<float, 2>(h, m) : launch_gc_t<double, 2>(h, m);
    return fail(HPHI_ERR_UNSUPPORTED, "SpinGC H*v takes one real or one complex vector per call");
}

// ------------------------------------------------------- diagonal, trace --

__device__ __forceinline__ double gc_diag_at(const GcDiagDev *d, int nd, const double *hz, int n, uint64_t x)
{
    double s = 0.0;
    for (int b = 0; b < nd; ++b) {
        const uint32_t m = d[b].mask, tb = (uint32_t)x & m;
        s += (tb == 0u || tb == m) ? d[b].jz4 : -d[b].jz4;
    }
    if (hz)
        for (int i = 0; i < n; ++i) s -= hz[i] * (((x >> i) & 1ull) ? 0.5 : -0.5);
    return s;
}

__global__ __launch_bounds__(kBlock) void k_gc_diag(const GcDiagDev *d, int nd, const double *hz, int n,
                                                    int64_t dim, double *out)
{
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += (int64_t)gridDim.x * blockDim.x)
        out[x] = gc_diag_at(d, nd, hz, n, (uint64_t)x);
}

__global__ __launch_bounds__(kBlock) void k_gc_trace(const GcDiagDev *d, int nd, const double *hz, int n,
                                                     int64_t dim, Reduce red)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[1];
    double acc = 0.0;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += (int64_t)gridDim.x * blockDim.x)
        acc += gc_diag_at(d, nd, hz, n, (uint64_t)x);
    double vv[1] = {acc};
    block_sum<1>(vv, sh);
    if (threadIdx.x == 0) blk[0] = vv[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

static unsigned gc_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, 2048)); }

int launch_gc_diag(hphi_ham *h, double *out, hipStream_t st)
{
    const hphi_basis *b = h->basis;
    hipLaunchKernelGGL(k_gc_diag, dim3(gc_grid(b->dim)), dim3(kBlock), 0, st, h->gc_diag.as<GcDiagDev>(),
                       h->gc_ndiag, h->gc_has_hz ? h->gc_hz.as<double>() : nullptr, b->n_sites, b->dim, out);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_gc_trace(hphi_ham *h, Reduce red, hipStream_t st)
{
    const hphi_basis *b = h->basis;
    hipLaunchKernelGGL(k_gc_trace, dim3(gc_grid(b->dim)), dim3(kBlock), 0, st, h->gc_diag.as<GcDiagDev>(),
                       h->gc_ndiag, h->gc_has_hz ? h->gc_hz.as<double>() : nullptr, b->n_sites, b->dim, red);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// b[x] = (sum_l phase_l S^z_l(x)) psi[x] on the full space.
__global__ void k_gc_szq(int64_t dim, int n_sites, const double *phase, const double *psi, double *b)
{
    __shared__ double ph[128];
    for (int i = threadIdx.x; i < 2 * n_sites; i += blockDim.x) ph[i] = phase[i];
    __syncthreads();
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < dim; x += (int64_t)gridDim.x * blockDim.x) {
        double re = 0.0, im = 0.0;
        for (int l = 0; l < n_sites; ++l) {
            const double sz = ((x >> l) & 1) ? 0.5 : -0.5;
            re += sz * ph[2 * l];
            im += sz * ph[2 * l + 1];
        }
        const double p = psi[x];
        b[2 * x] = re * p;
        b[2 * x + 1] = im * p;
    }
}

int launch_gc_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st)
{
    const hphi_basis *bs = h->basis;
    hipLaunchKernelGGL(k_gc_szq, dim3(gc_grid(bs->dim)), dim3(kBlock), 0, st, bs->dim, bs->n_sites, phase_dev,
                       static_cast<const double *>(psi), static_cast<double *>(b));
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

__global__ void k_gc_states(int64_t first, int64_t count, uint64_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint64_t)(first + i);
}

__global__ void k_gc_rank(const uint64_t *s, int64_t n, int64_t dim, int64_t *idx)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        idx[i] = s[i] < (uint64_t)dim ? (int64_t)s[i] : -1;
}

int launch_gc_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out, hipStream_t st)
{
    if (count <= 0) return HPHI_OK;
    hipLaunchKernelGGL(k_gc_states, dim3(gc_grid(count)), dim3(kBlock), 0, st, first, count, out);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_gc_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx, hipStream_t st)
{
    if (n <= 0) return HPHI_OK;
    hipLaunchKernelGGL(k_gc_rank, dim3(gc_grid(n)), dim3(kBlock), 0, st, states, n, b->dim, idx);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

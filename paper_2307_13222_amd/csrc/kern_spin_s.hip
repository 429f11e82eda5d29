// Spin-S Heisenberg H*v with total S^z conserved (keyword 2S of the HPhi
// update paper, Sec. 4.1, "Remarks on the keyword model"):
//   H = sum_b [jz S^z_i S^z_j + jxy/2 (S^+_i S^-_j + S^-_i S^+_j)]
//       - sum_i hz_i S^z_i + sum_i d_i (S^z_i)^2.
// Site i holds m_i = S^z_i + S in a b-bit field; S^+_i S^-_j adds 1 to
// field i and takes 1 from field j, so the target configuration is
// x + 2^(i b) - 2^(j b), ranked by the sector's split two-level table. The
// ladder amplitudes sqrt(S(S+1) - s(s+-1)) come from a table over m. One
// thread per row, the epilogue and FP64 dots of the caller fused.
#include "kern_common.h"
#include "row_finish.h"

namespace hphi {

struct SpinSBondDev {
    int32_t i, j;
    double jz, jxy2;   // jxy / 2
};

struct SpinSKArgs {
    const uint64_t *states;
    int64_t dim;
    const uint32_t *hi_off, *lo_rank;
    int bits, lo_bits, two_s, n_sites;
    const SpinSBondDev *bonds;
    int nb;
    const double *hz, *dion;
    double amp_up[8], amp_dn[8];   // <m+1|S^+|m>, <m-1|S^-|m>
    double s;                      // S
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

// BOND_LDS: the bond records staged in dynamic LDS (wave-uniform reads).
// The ladder terms run in batches of eight slots (slot 2k: S^+_i S^-_j of
// bond k, slot 2k + 1: S^-_i S^+_j): targets first, then their rank-table
// loads, then the gathers, all eight in flight at each level; a slot that
// does not apply gathers this row's own element with coefficient 0.
template <typename S, int NV, bool DOTS, bool BOND_LDS>
__global__ __launch_bounds__(256) void k_spin_s_hv(SpinSKArgs a)
{
    extern __shared__ SpinSBondDev s_bonds[];
    __shared__ double sh_red[2 * NV * 4 > 16 ? 2 * NV * 4 : 16];
    __shared__ double sh_blk[2 * NV];
    const SpinSBondDev *bonds = a.bonds;
    if constexpr (BOND_LDS) {
        for (int k = threadIdx.x; k < a.nb; k += blockDim.x) s_bonds[k] = a.bonds[k];
        __syncthreads();
        bonds = s_bonds;
    }
    const S *__restrict__ v = static_cast<const S *>(a.v);
    const EpiArgs<S> ep{static_cast<S *>(a.w), static_cast<const S *>(a.u), static_cast<S *>(a.acc_out),
                        static_cast<S *>(a.raw_out), a.coef, a.coef_cplx, a.dot_raw};
    RowFinish<S, NV, DOTS> fin;
    fin.init(ep);
    const uint64_t dmask = (1ull << a.bits) - 1ull, lomask = (1ull << a.lo_bits) - 1ull;
    const int nslot = 2 * a.nb;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.dim; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = a.states[r];
        double dg = 0.0;
        S hv[NV], me[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            hv[j] = (S)0;
            me[j] = v[(size_t)r * NV + j];
        }
        for (int k = 0; k < a.nb; ++k) {
            const SpinSBondDev bd = bonds[k];
            const int mi = (int)((x >> (bd.i * a.bits)) & dmask), mj = (int)((x >> (bd.j * a.bits)) & dmask);
            dg += bd.jz * ((double)mi - a.s) * ((double)mj - a.s);
        }
        constexpr int B = 8;
        for (int s0 = 0; s0 < nslot; s0 += B) {
            uint64_t y[B];
            double cf[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const int sl = s0 + t;
                y[t] = x;
                cf[t] = 0.0;
                if (sl < nslot) {
                    const SpinSBondDev bd = bonds[sl >> 1];
                    const int si = bd.i * a.bits, sj = bd.j * a.bits;
                    const int mi = (int)((x >> si) & dmask), mj = (int)((x >> sj) & dmask);
                    if (!(sl & 1)) {
                        if (bd.jxy2 != 0.0 && mi < a.two_s && mj > 0) {
                            y[t] = x + (1ull << si) - (1ull << sj);
                            cf[t] = bd.jxy2 * a.amp_up[mi] * a.amp_dn[mj];
                        }
                    } else if (bd.jxy2 != 0.0 && mi > 0 && mj < a.two_s) {
                        y[t] = x - (1ull << si) + (1ull << sj);
                        cf[t] = bd.jxy2 * a.amp_dn[mi] * a.amp_up[mj];
                    }
                }
            }
            uint32_t ho[B], lr[B];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                ho[t] = a.hi_off[y[t] >> a.lo_bits];
                lr[t] = a.lo_rank[y[t] & lomask];
            }
            S g[B][NV];
#pragma unroll
            for (int t = 0; t < B; ++t) {
                const size_t c = (size_t)ho[t] + lr[t];
#pragma unroll
                for (int j = 0; j < NV; ++j) g[t][j] = v[c * NV + j];
            }
#pragma unroll
            for (int t = 0; t < B; ++t)
#pragma unroll
                for (int j = 0; j < NV; ++j) hv[j] += (S)cf[t] * g[t][j];
        }
        for (int i = 0; i < a.n_sites && (a.hz || a.dion); ++i) {
            const double sz = (double)((x >> (i * a.bits)) & dmask) - a.s;
            if (a.hz) dg -= a.hz[i] * sz;
            if (a.dion) dg += a.dion[i] * sz * sz;
        }
#pragma unroll
        for (int j = 0; j < NV; ++j) hv[j] += (S)dg * me[j];
        fin.apply(hv, me, (size_t)r, ep);
    }
    fin.reduce(a.red, sh_red, sh_blk);
}

static SpinSKArgs spin_s_args(hphi_ham *h)
{
    const SpinSTables &t = h->basis->ss;
    SpinSKArgs a{};
    a.states = t.d_states.as<uint64_t>();
    a.dim = h->basis->dim;
    a.hi_off = t.d_hi_off32.as<uint32_t>();
    a.lo_rank = t.d_lo_rank.as<uint32_t>();
    a.bits = t.bits;
    a.lo_bits = t.lo_bits;
    a.two_s = t.two_s;
    a.n_sites = h->basis->n_sites;
    a.bonds = h->s_dbonds.as<SpinSBondDev>();
    a.nb = (int)h->sbonds.size();
    a.hz = h->s_hz.empty() ? nullptr : h->s_dhz.as<double>();
    a.dion = h->s_dion.empty() ? nullptr : h->s_ddion.as<double>();
    a.s = 0.5 * t.two_s;
    for (int m = 0; m <= t.two_s && m < 8; ++m) {
        const double sz = m - a.s, ss = a.s * (a.s + 1.0);
        a.amp_up[m] = m < t.two_s ? std::sqrt(ss - sz * (sz + 1.0)) : 0.0;
        a.amp_dn[m] = m > 0 ? std::sqrt(ss - sz * (sz - 1.0)) : 0.0;
    }
    return a;
}

static unsigned spin_s_grid(int64_t n, int threads)
{
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + threads - 1) / threads, 4096));
}

template <typename S, int NV>
static int launch_spin_s_t(hphi_ham *h, const MultArgs &m)
{
    SpinSKArgs a = spin_s_args(h);
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
    const unsigned grid = spin_s_grid(a.dim, 256);
    const size_t lds = sizeof(SpinSBondDev) * (size_t)a.nb;
    const bool bl = lds <= 32 * 1024;
    auto go = [&](auto kern) {
        if (bl) hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), bl ? lds : 0, m.stream, a);
    };
    if (a.nd) bl ? go(k_spin_s_hv<S, NV, true, true>) : go(k_spin_s_hv<S, NV, true, false>);
    else bl ? go(k_spin_s_hv<S, NV, false, true>) : go(k_spin_s_hv<S, NV, false, false>);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_spin_s_mult(hphi_ham *h, const MultArgs &m)
{
    if (m.lz || m.lz_q) return fail(HPHI_ERR_UNSUPPORTED, "spin-S: no fused Lanczos update");
    if (m.ld > 0 && m.ld != h->basis->dim) return fail(HPHI_ERR_UNSUPPORTED, "spin-S: no row pitch");
    if (m.v == m.w) return fail(HPHI_ERR_INVALID_ARG, "spin-S H*v: w may not alias v");
    const int nv = m.nvec * dtype_lanes(m.dtype);
    const bool f32 = dtype_is_f32(m.dtype);
    if (nv == 1) return f32 ? launch_spin_s_t<float, 1>(h, m) : launch_spin_s_t<double, 1>(h, m);
    if (nv == 2) return f32 ? launch_spin_s_t<float, 2>(h, m) : launch_spin_s_t<double, 2>(h, m);
    return fail(HPHI_ERR_UNSUPPORTED, "spin-S H*v takes one real or one complex vector per call");
}

// ------------------------------------------------- diagonal, trace, S^z(q) --

__device__ __forceinline__ double spin_s_diag_at(const SpinSKArgs &a, uint64_t x)
{
    const uint64_t dmask = (1ull << a.bits) - 1ull;
    double dg = 0.0;
    for (int k = 0; k < a.nb; ++k) {
        const int mi = (int)((x >> (a.bonds[k].i * a.bits)) & dmask), mj = (int)((x >> (a.bonds[k].j * a.bits)) & dmask);
        dg += a.bonds[k].jz * ((double)mi - a.s) * ((double)mj - a.s);
    }
    for (int i = 0; i < a.n_sites && (a.hz || a.dion); ++i) {
        const double sz = (double)((x >> (i * a.bits)) & dmask) - a.s;
        if (a.hz) dg -= a.hz[i] * sz;
        if (a.dion) dg += a.dion[i] * sz * sz;
    }
    return dg;
}

__global__ __launch_bounds__(kBlock) void k_spin_s_diag(SpinSKArgs a, double *out)
{
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.dim; r += (int64_t)gridDim.x * blockDim.x)
        out[r] = spin_s_diag_at(a, a.states[r]);
}

__global__ __launch_bounds__(kBlock) void k_spin_s_trace(SpinSKArgs a, Reduce red)
{
    __shared__ double sh[kBlock / kWave];
    __shared__ double blk[1];
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.dim; r += (int64_t)gridDim.x * blockDim.x)
        acc += spin_s_diag_at(a, a.states[r]);
    double vv[1] = {acc};
    block_sum<1>(vv, sh);
    if (threadIdx.x == 0) blk[0] = vv[0];
    __syncthreads();
    grid_finish(blk, 1, red, sh);
}

// b[r] = (sum_l phase_l S^z_l(x_r)) psi[r], S^z_l = m_l - S
__global__ void k_spin_s_szq(SpinSKArgs a, const double *phase, const double *psi, double *b)
{
    __shared__ double ph[128];
    for (int i = threadIdx.x; i < 2 * a.n_sites; i += blockDim.x) ph[i] = phase[i];
    __syncthreads();
    const uint64_t dmask = (1ull << a.bits) - 1ull;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.dim; r += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = a.states[r];
        double re = 0.0, im = 0.0;
        for (int l = 0; l < a.n_sites; ++l) {
            const double sz = (double)((x >> (l * a.bits)) & dmask) - a.s;
            re += sz * ph[2 * l];
            im += sz * ph[2 * l + 1];
        }
        b[2 * r] = re * psi[r];
        b[2 * r + 1] = im * psi[r];
    }
}

int launch_spin_s_diag(hphi_ham *h, double *out, hipStream_t st)
{
    const SpinSKArgs a = spin_s_args(h);
    hipLaunchKernelGGL(k_spin_s_diag, dim3(spin_s_grid(a.dim, kBlock)), dim3(kBlock), 0, st, a, out);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_spin_s_trace(hphi_ham *h, Reduce red, hipStream_t st)
{
    const SpinSKArgs a = spin_s_args(h);
    hipLaunchKernelGGL(k_spin_s_trace, dim3(std::min(spin_s_grid(a.dim, kBlock), 2048u)), dim3(kBlock), 0, st, a,
                       red);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_spin_s_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st)
{
    const SpinSKArgs a = spin_s_args(h);
    hipLaunchKernelGGL(k_spin_s_szq, dim3(spin_s_grid(a.dim, kBlock)), dim3(kBlock), 0, st, a, phase_dev,
                       static_cast<const double *>(psi), static_cast<double *>(b));
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

__global__ void k_spin_s_states(const uint64_t *states, int64_t first, int64_t count, uint64_t *out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = states[first + i];
}

// rank of each configuration; -1 outside the sector (a digit above 2S, a
// wrong digit sum, bits beyond the N fields)
__global__ void k_spin_s_rank(const uint64_t *s, int64_t n, const uint32_t *hi_off, const uint32_t *lo_rank,
                              const uint64_t *states, int64_t dim, int bits, int lo_bits, int n_sites, int two_s,
                              int64_t *idx)
{
    const uint64_t dmask = (1ull << bits) - 1ull, lomask = (1ull << lo_bits) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = s[i];
        bool ok = n_sites * bits >= 64 || (x >> (n_sites * bits)) == 0ull;
        for (int l = 0; l < n_sites && ok; ++l)
            if ((int)((x >> (l * bits)) & dmask) > two_s) ok = false;
        int64_t r = -1;
        if (ok) {
            const uint32_t lr = lo_rank[x & lomask];
            const int64_t c = (int64_t)hi_off[x >> lo_bits] + lr;
            // a configuration of the wrong digit sum lands on another
            // state's index: accept it only if that state is x itself
            if (lr != 0xFFFFFFFFu && c >= 0 && c < dim && states[c] == x) r = c;
        }
        idx[i] = r;
    }
}

int launch_spin_s_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out, hipStream_t st)
{
    if (count <= 0) return HPHI_OK;
    hipLaunchKernelGGL(k_spin_s_states, dim3(spin_s_grid(count, kBlock)), dim3(kBlock), 0, st,
                       b->ss.d_states.as<uint64_t>(), first, count, out);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_spin_s_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx, hipStream_t st)
{
    if (n <= 0) return HPHI_OK;
    const SpinSTables &t = b->ss;
    hipLaunchKernelGGL(k_spin_s_rank, dim3(spin_s_grid(n, kBlock)), dim3(kBlock), 0, st, states, n,
                       t.d_hi_off32.as<uint32_t>(), t.d_lo_rank.as<uint32_t>(), t.d_states.as<uint64_t>(), b->dim,
                       t.bits, t.lo_bits, b->n_sites, t.two_s, idx);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

// Spin-1/2 XXZ H*v on an implicit sector basis: no state list is stored
// (at 36 sites and S^z = 0 the list alone would be 72.6 GB). A row index r
// is mapped back to its configuration through the same split two-level
// table that ranks it: the high pattern h is the block with
// hi_off[h] <= r < hi_off[h + 1], and the low pattern is entry
// r - hi_off[h] of the ascending list of n_lo-bit patterns with
// n_pop - popcount(h) set bits. Indices are 64-bit throughout.
//
// Rows are handed out in contiguous runs of one workgroup; thread 0 finds
// the block of the run's first row by binary search, and each lane advances
// from there (a run crosses a block boundary only near the sector's sparse
// edges). Matrix elements and the fused epilogue / FP64 dots are those of
// the materialized kernel (HPhi update paper Sec. 3.2 Heisenberg model).
#include "kern_common.h"

namespace hphi {

struct BigKArgs {
    int64_t dim;
    const uint64_t *hi_off;      // 2^n_hi + 1
    const uint32_t *lo_rank;     // 2^n_lo
    const uint32_t *lo_list;     // patterns grouped by popcount
    const uint32_t *lo_list_off; // n_lo + 2
    int n_lo, n_hi, n_pop;
    const SpinBondDev *bonds;
    int nb;
    const double *hz;
    int n_sites;
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    const double *coef;
    int nd;
    int dot_raw;
    Reduce red;
};

template <typename S, bool DOTS>
__global__ __launch_bounds__(kBlock) void k_spin_hv_implicit(BigKArgs a)
{
    __shared__ double sh_red[kBlock / kWave * 2];
    __shared__ double sh_blk[2];
    __shared__ uint64_t s_h0;
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *__restrict__ accp = static_cast<S *>(a.acc_out);
    double c1 = 1.0, c2 = 0.0;
    if (a.coef) {
        c1 = a.coef[0];
        c2 = a.coef[1];
    }
    const S c1s = (S)c1, c2s = (S)c2;
    const uint64_t lomask = (uint64_t(1) << a.n_lo) - 1;
    const uint64_t nh = uint64_t(1) << a.n_hi;
    double d0 = 0.0, d1 = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.dim; base += (int64_t)gridDim.x * blockDim.x) {
        __syncthreads();
        if (threadIdx.x == 0) {
            // last h with hi_off[h] <= base
            uint64_t lo = 0, hi = nh;
            while (hi - lo > 1) {
                const uint64_t mid = (lo + hi) >> 1;
                if (a.hi_off[mid] <= (uint64_t)base) lo = mid; else hi = mid;
            }
            s_h0 = lo;
        }
        __syncthreads();
        const int64_t r = base + threadIdx.x;
        if (r >= a.dim) continue;
        uint64_t h = s_h0;
        while (a.hi_off[h + 1] <= (uint64_t)r) ++h;
        const uint64_t j = (uint64_t)r - a.hi_off[h];
        const int k = a.n_pop - __popcll(h);
        const uint64_t x = (h << a.n_lo) | (uint64_t)a.lo_list[a.lo_list_off[k] + j];
        S acc = (S)0, diag = (S)0;
        for (int b = 0; b < a.nb; ++b) {
            const uint64_t m = a.bonds[b].mask;
            const uint64_t t = x & m;
            const S jz4 = (S)a.bonds[b].jz4;
            if (t == 0 || t == m) {
                diag += jz4;
            } else {
                diag -= jz4;
                const uint64_t y = x ^ m;
                const uint64_t idx = a.hi_off[y >> a.n_lo] + a.lo_rank[y & lomask];
                acc += (S)a.bonds[b].jxy2 * v[idx];
            }
        }
        if (a.hz)
            for (int i = 0; i < a.n_sites; ++i) diag -= (S)a.hz[i] * (((x >> i) & 1) ? (S)0.5 : (S)-0.5);
        const S me = v[r];
        const S hv = acc + diag * me;
        S out = c1s * hv;
        if (u) out += c2s * u[r];
        w[r] = out;
        if (accp) accp[r] += out;
        if constexpr (DOTS) {
            const double o = a.dot_raw ? (double)hv : (double)out;
            d0 += (double)me * o;
            d1 += o * o;
        }
    }
    if constexpr (DOTS) {
        double vals[2] = {d0, d1};
        block_sum<2>(vals, sh_red);
        if (threadIdx.x == 0) {
            sh_blk[0] = vals[0];
            sh_blk[1] = vals[1];
        }
        __syncthreads();
        grid_finish(sh_blk, 2, a.red, sh_red);
    }
}

int launch_spin_mult_implicit(hphi_ham *h, const MultArgs &m)
{
    const hphi_basis *b = h->basis;
    const Species &s = b->sp[0];
    const int mode = spin_split_mode(h, true);
    const bool apart = m.v != m.w && (!m.u || m.u != m.w) && (!m.acc || m.acc != m.w);
    if (m.nvec * dtype_lanes(m.dtype) != 1) {
        // several lanes per state (vector blocks, complex vectors): the
        // block-staged product only
        if (mode == 2 && !m.dots && !m.cocg && apart) {
            int done = 0;
            HPHI_TRY(launch_spin_blk(h, m, &done));
            if (done) return HPHI_OK;
        }
        return fail(HPHI_ERR_UNSUPPORTED,
                    "implicit-basis H*v: several lanes per state need the block-staged product (schedule spin_split 2 "
                    "or 3, no fused dots)");
    }
    BigKArgs a{};
    a.dim = s.dim;
    a.hi_off = s.d_hi_off.as<uint64_t>();
    a.lo_rank = s.d_lo_rank.as<uint32_t>();
    a.lo_list = s.d_lo_list.as<uint32_t>();
    a.lo_list_off = s.d_lo_list_off.as<uint32_t>();
    a.n_lo = s.n_lo;
    a.n_hi = s.n_hi;
    a.n_pop = s.n_pop;
    a.bonds = h->d_bonds.as<SpinBondDev>();
    a.nb = h->n_bonds;
    a.hz = h->has_field ? h->d_hz.as<double>() : nullptr;
    a.n_sites = b->n_sites;
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.coef = m.coef;
    a.nd = m.dots;
    a.dot_raw = m.dot_raw;
    a.red = m.red;
    const int ncu = b->ctx->n_cu > 0 ? b->ctx->n_cu : 256;
    int64_t need = (s.dim + kBlock - 1) / kBlock;
    int64_t cap = (int64_t)ncu * h->sched_cfg.spin_per_cu;
    if (cap > kMaxGrid) cap = kMaxGrid;
    const int grid = (int)(need < cap ? need : cap);
    const bool f32 = dtype_is_f32(m.dtype);
    // split product (schedule spin_split): the bonds with an end in the low
    // half and the fields here into w, then the high-half bonds and the
    // caller's epilogue in slab order (their gathers are contiguous runs
    // of one block of the same class)
    bool split = mode != 0 && !m.dots && !m.cocg && apart;
    if (split && mode == 2) {
        int done = 0;
        HPHI_TRY(launch_spin_blk(h, m, &done));
        if (done) return HPHI_OK;
    }
    if (split) {
        HPHI_TRY(spin_split_tables(h));
        split = h->split.n_hi_bonds > 0 && h->split.n_hi_bonds <= kMaxHiBonds;
    }
    if (split) {
        a.bonds = h->split.rest.as<SpinBondDev>();
        a.nb = h->split.n_rest;
        a.u = nullptr;
        a.acc_out = nullptr;
        a.coef = nullptr;
        a.nd = 0;
        if (f32) hipLaunchKernelGGL((k_spin_hv_implicit<float, false>), dim3(grid), dim3(kBlock), 0, m.stream, a);
        else hipLaunchKernelGGL((k_spin_hv_implicit<double, false>), dim3(grid), dim3(kBlock), 0, m.stream, a);
        HPHI_HIP(hipGetLastError());
        return launch_spin_hi_pass(h, m);
    }
    if (a.nd) {
        if (f32) hipLaunchKernelGGL((k_spin_hv_implicit<float, true>), dim3(grid), dim3(kBlock), 0, m.stream, a);
        else hipLaunchKernelGGL((k_spin_hv_implicit<double, true>), dim3(grid), dim3(kBlock), 0, m.stream, a);
    } else {
        if (f32) hipLaunchKernelGGL((k_spin_hv_implicit<float, false>), dim3(grid), dim3(kBlock), 0, m.stream, a);
        else hipLaunchKernelGGL((k_spin_hv_implicit<double, false>), dim3(grid), dim3(kBlock), 0, m.stream, a);
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

// Spin-1/2 XXZ H*v on the S^z-conserved basis (Heisenberg/XXZ model of the
// HPhi update paper, Sec. 3.2 and the Spin model keyword of Sec. 4.1).
//
// Gather formulation, one thread per output state x (row owner, no atomics):
//   w[x] = diag(x) v[x] + sum_{bonds b antiparallel in x} (Jxy_b / 2) v[rank(x ^ m_b)]
//   diag(x) = sum_b (Jz_b / 4) (+1 parallel, -1 antiparallel) - sum_i h_i S^z_i
// rank() is the split two-level table hi_off[y >> n_lo] + lo_rank[y & mask],
// staged in LDS when it fits. A block of NV real lanes per state (NV = 1 for
// a real vector, 2 for one complex vector, 32 for 16 complex vectors) is
// stored interleaved, so one gather moves NV * sizeof(S) contiguous bytes and
// the index work is paid once for all lanes.
#include "kern_common.h"

namespace hphi {

struct SpinKArgs {
    const uint32_t *states;
    int64_t dim;
    const SpinBondDev *bonds;
    int nb;
    const double *hz;
    int n_sites;
    const uint32_t *lo_rank;
    const uint32_t *hi_off;
    int n_lo, n_hi;
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    const double *coef;
    int nd;
    int dot_raw;   // dots of H v itself (1) or of the epilogue output (0)
    Reduce red;
    int coef_cplx;
    void *raw_out;   // optional: H v itself (before the epilogue), same layout as w
    CgDev *cocg;     // optional (NV = 2 with dots): COCG mu and alpha step
};

// Load NV contiguous scalars at p (p aligned to min(16, NV * sizeof(S))).
template <typename S, int NV>
__device__ __forceinline__ void load_lanes(const S *__restrict__ p, S (&o)[NV])
{
    constexpr int B = NV * (int)sizeof(S);
    if constexpr (B >= 16) {
        const float4 *q = reinterpret_cast<const float4 *>(p);
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            float4 t = q[k];
            S *d = o + k * (16 / (int)sizeof(S));
            __builtin_memcpy(d, &t, 16);
        }
    } else if constexpr (B == 8) {
        float2 t = *reinterpret_cast<const float2 *>(p);
        __builtin_memcpy(o, &t, 8);
    } else {
        o[0] = p[0];
    }
}

template <typename S, int NV>
__device__ __forceinline__ void store_lanes(S *__restrict__ p, const S (&o)[NV])
{
    constexpr int B = NV * (int)sizeof(S);
    if constexpr (B >= 16) {
        float4 *q = reinterpret_cast<float4 *>(p);
#pragma unroll
        for (int k = 0; k < B / 16; ++k) {
            float4 t;
            __builtin_memcpy(&t, o + k * (16 / (int)sizeof(S)), 16);
            q[k] = t;
        }
    } else if constexpr (B == 8) {
        float2 t;
        __builtin_memcpy(&t, o, 8);
        *reinterpret_cast<float2 *>(p) = t;
    } else {
        p[0] = o[0];
    }
}

// TAB: where rank() reads its tables. 0: global memory; 1: both 32-bit
// tables in LDS (kBlock threads); 2: hi_off (32-bit) and lo_rank narrowed
// to 16 bits in LDS (ranks below 65536), kSpinBigBlock threads, so tables
// of up to 96 KB (27 and 28 sites) sit in LDS at one workgroup per CU, and
// the tables of 23 to 26 sites leave 16 to 32 waves per CU (with 32-bit
// tables and kBlock threads the LDS held 8 to 16).
constexpr int kSpinBigBlock = 1024;
template <int TAB> constexpr int spin_block() { return TAB == 2 ? kSpinBigBlock : kBlock; }

// Narrowed-table kernels with fused dots on states of at most 16 bytes:
// registers for two 1024-thread workgroups per CU (8 waves per SIMD), as
// their LDS allows (the dots' FP64 accumulators would otherwise leave one).
template <int TAB, typename S, int NV, bool DOTS> constexpr int spin_min_waves()
{
    return (TAB == 2 && DOTS && NV * sizeof(S) <= 16) ? 8 : 1;
}

template <typename S, int NV, int TAB, bool DOTS>
__global__ __launch_bounds__(spin_block<TAB>(), (spin_min_waves<TAB, S, NV, DOTS>())) void k_spin_hv(SpinKArgs a)
{
    extern __shared__ uint32_t smem_tab[];
    __shared__ double sh_red[spin_block<TAB>() / kWave * 2 * 32];
    __shared__ double sh_blk[64];

    const uint32_t *lo = a.lo_rank;
    const uint32_t *hi = a.hi_off;
    const uint16_t *lo16 = nullptr;
    if constexpr (TAB == 1) {
        const int nl = 1 << a.n_lo, nh = 1 << a.n_hi;
        for (int i = threadIdx.x; i < nl; i += blockDim.x) smem_tab[i] = a.lo_rank[i];
        for (int i = threadIdx.x; i < nh; i += blockDim.x) smem_tab[nl + i] = a.hi_off[i];
        __syncthreads();
        lo = smem_tab;
        hi = smem_tab + nl;
    } else if constexpr (TAB == 2) {
        const int nl = 1 << a.n_lo, nh = 1 << a.n_hi;
        uint16_t *l16 = reinterpret_cast<uint16_t *>(smem_tab + nh);
        for (int i = threadIdx.x; i < nh; i += blockDim.x) smem_tab[i] = a.hi_off[i];
        for (int i = threadIdx.x; i < nl; i += blockDim.x) l16[i] = (uint16_t)a.lo_rank[i];
        __syncthreads();
        hi = smem_tab;
        lo16 = l16;
    }
    const uint32_t lomask = (1u << a.n_lo) - 1u;
    const int n_lo = a.n_lo;
    // rank of an in-sector configuration
    auto rank = [&](uint32_t y) -> uint32_t {
        if constexpr (TAB == 2) return hi[y >> n_lo] + (uint32_t)lo16[y & lomask];
        else return hi[y >> n_lo] + lo[y & lomask];
    };
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

    constexpr int ND = DOTS ? NV : 1;
    CgDev *const cgp = (DOTS && NV == 2) ? a.cocg : nullptr;
    const cd zs = cgp ? cgp->zs : cd{0.0, 0.0};
    double d0[ND], d1[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) d0[j] = d1[j] = 0.0;

    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < a.dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = a.states[r];
        S acc[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) acc[j] = (S)0;
        S diag = (S)0;
        if constexpr (NV <= 4) {
            // narrow lanes: eight bonds per batch, their targets first, then
            // all eight gathers in flight, then the sums in bond order (an
            // antiparallel-free slot re-reads this state and adds exactly +0)
            constexpr int BB = 8;
            for (int b0 = 0; b0 < a.nb; b0 += BB) {
                uint32_t idx[BB];
                S cf[BB];
#pragma unroll
                for (int k = 0; k < BB; ++k) {
                    idx[k] = (uint32_t)r;
                    cf[k] = (S)0;
                    const int b = b0 + k;
                    if (b < a.nb) {
                        const uint32_t m = (uint32_t)a.bonds[b].mask;
                        const uint32_t t = x & m;
                        const S jz4 = (S)a.bonds[b].jz4;
                        if (t == 0u || t == m) {
                            diag += jz4;
                        } else {
                            diag -= jz4;
                            const uint32_t y = x ^ m;
                            idx[k] = rank(y);
                            cf[k] = (S)a.bonds[b].jxy2;
                        }
                    }
                }
                S nv[BB][NV];
#pragma unroll
                for (int k = 0; k < BB; ++k) load_lanes<S, NV>(v + (size_t)idx[k] * NV, nv[k]);
#pragma unroll
                for (int k = 0; k < BB; ++k)
#pragma unroll
                    for (int j = 0; j < NV; ++j) acc[j] += cf[k] * nv[k][j];
            }
        } else {
            for (int b = 0; b < a.nb; ++b) {
                const uint32_t m = (uint32_t)a.bonds[b].mask;
                const uint32_t t = x & m;
                const S jz4 = (S)a.bonds[b].jz4;
                if (t == 0u || t == m) {
                    diag += jz4;
                } else {
                    diag -= jz4;
                    const uint32_t y = x ^ m;
                    const uint32_t idx = rank(y);
                    const S cf = (S)a.bonds[b].jxy2;
                    S nv[NV];
                    load_lanes<S, NV>(v + (size_t)idx * NV, nv);
#pragma unroll
                    for (int j = 0; j < NV; ++j) acc[j] += cf * nv[j];
                }
            }
        }
        if (a.hz) {
            for (int i = 0; i < a.n_sites; ++i)
                diag -= (S)a.hz[i] * (((x >> i) & 1u) ? (S)0.5 : (S)-0.5);
        }
        S me[NV];
        load_lanes<S, NV>(v + (size_t)r * NV, me);
        S hv[NV], out[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) hv[j] = acc[j] + diag * me[j];
        if (a.coef_cplx) {
            S uu[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) uu[j] = (S)0;
            if (u) load_lanes<S, NV>(u + (size_t)r * NV, uu);
            epilogue_r<S, NV>(hv, uu, u != nullptr, 1, a.coef, out);
        } else {
#pragma unroll
            for (int j = 0; j < NV; ++j) out[j] = c1s * hv[j];
            if (u) {
                S uu[NV];
                load_lanes<S, NV>(u + (size_t)r * NV, uu);
#pragma unroll
                for (int j = 0; j < NV; ++j) out[j] += c2s * uu[j];
            }
        }
        store_lanes<S, NV>(w + (size_t)r * NV, out);
        if (a.raw_out) store_lanes<S, NV>(static_cast<S *>(a.raw_out) + (size_t)r * NV, hv);
        if (accp) {
            S aa[NV];
            load_lanes<S, NV>(accp + (size_t)r * NV, aa);
#pragma unroll
            for (int j = 0; j < NV; ++j) aa[j] += out[j];
            store_lanes<S, NV>(accp + (size_t)r * NV, aa);
        }
        if constexpr (DOTS) {
            bool cg_done = false;
            if constexpr (NV == 2) {
                if (cgp) {
                    // COCG mu term p^T (z_s p - H p) of this state
                    const cd pv = {(double)me[0], (double)me[1]};
                    const cd t = cmul(pv, csub(cmul(zs, pv), cd{(double)hv[0], (double)hv[1]}));
                    d0[0] += t.re;
                    d0[1] += t.im;
                    cg_done = true;
                }
            }
            if (!cg_done) {
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const double o = a.dot_raw ? (double)hv[j] : (double)out[j];
                    d0[j] += (double)me[j] * o;
                    d1[j] += o * o;
                }
            }
        }
    }
    if constexpr (DOTS) {
        // per-lane sums: across each wave with shuffles (the accumulators
        // stay in registers: every index is a compile-time constant), then
        // over the block's waves in wave order
        const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            const double s0 = wave_sum(d0[j]), s1 = wave_sum(d1[j]);
            if (lane == 0) {
                sh_red[wid * 2 * NV + j] = s0;
                sh_red[wid * 2 * NV + NV + j] = s1;
            }
        }
        __syncthreads();
        if (threadIdx.x < 2 * NV) {
            double t = 0.0;
            for (int w2 = 0; w2 < nw; ++w2) t += sh_red[w2 * 2 * NV + threadIdx.x];
            sh_blk[threadIdx.x] = t;
        }
        __syncthreads();
        if (grid_finish(sh_blk, 2 * NV, a.red, sh_red) && cgp && threadIdx.x == 0)
            cocg_alpha_step(cgp, {a.red.result[0], a.red.result[1]});
    }
}

template <typename S, int NV, int LDS>
static void launch_spin_d(const SpinKArgs &a, int grid, size_t lds_bytes, hipStream_t st)
{
    constexpr int BS = spin_block<LDS>();
    if constexpr (LDS == 2) {
        // the launcher picks these tables for fused dots only up to 32 B
        // per state (the FP64 accumulators of wider states do not fit the
        // registers of a 1024-thread workgroup)
        if constexpr (NV * sizeof(S) <= 32) {
            if (a.nd) {
                hipFuncSetAttribute((const void *)k_spin_hv<S, NV, 2, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
                hipLaunchKernelGGL((k_spin_hv<S, NV, 2, true>), dim3(grid), dim3(BS), lds_bytes, st, a);
                return;
            }
        }
        hipFuncSetAttribute((const void *)k_spin_hv<S, NV, 2, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds_bytes);
        hipLaunchKernelGGL((k_spin_hv<S, NV, 2, false>), dim3(grid), dim3(BS), lds_bytes, st, a);
        return;
    } else if (a.nd) {
        if (LDS) hipFuncSetAttribute((const void *)k_spin_hv<S, NV, LDS, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        hipLaunchKernelGGL((k_spin_hv<S, NV, LDS, true>), dim3(grid), dim3(BS), lds_bytes, st, a);
    } else {
        if (LDS) hipFuncSetAttribute((const void *)k_spin_hv<S, NV, LDS, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        hipLaunchKernelGGL((k_spin_hv<S, NV, LDS, false>), dim3(grid), dim3(BS), lds_bytes, st, a);
    }
}

template <typename S, int NV>
static int launch_spin_t(const SpinKArgs &a, int tab, int grid, size_t lds_bytes, hipStream_t st)
{
    if constexpr (NV * sizeof(S) <= 128) {
        if (tab == 2) {
            launch_spin_d<S, NV, 2>(a, grid, lds_bytes, st);
            HPHI_HIP(hipGetLastError());
            return HPHI_OK;
        }
    }
    if (tab == 2) return fail(HPHI_ERR_UNSUPPORTED, "spin H*v: narrowed tables with %d-byte states", (int)(NV * sizeof(S)));
    if (tab == 1) launch_spin_d<S, NV, 1>(a, grid, lds_bytes, st);
    else launch_spin_d<S, NV, 0>(a, grid, 0, st);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

template <typename S>
static int launch_spin_nv(int nv, const SpinKArgs &a, int lds, int grid, size_t lds_bytes,
                          hipStream_t st)
{
    switch (nv) {
    case 1: return launch_spin_t<S, 1>(a, lds, grid, lds_bytes, st);
    case 2: return launch_spin_t<S, 2>(a, lds, grid, lds_bytes, st);
    case 4: return launch_spin_t<S, 4>(a, lds, grid, lds_bytes, st);
    case 8: return launch_spin_t<S, 8>(a, lds, grid, lds_bytes, st);
    case 16: return launch_spin_t<S, 16>(a, lds, grid, lds_bytes, st);
    case 32: return launch_spin_t<S, 32>(a, lds, grid, lds_bytes, st);
    }
    return fail(HPHI_ERR_UNSUPPORTED, "spin H*v: %d real lanes per state (supported 1,2,4,8,16,32)", nv);
}

// The stored-list kernel runs for a materialized basis with 32-bit states
// unless the schedule asks for the implicit one.
bool spin_stored_path(const hphi_ham *h)
{
    const Species &s = h->basis->sp[0];
    return s.materialized() && s.state_bytes == 4 && s.d_hi_off32.p && !h->sched_cfg.spin_implicit;
}

int spin_split_mode(const hphi_ham *h, bool implicit)
{
    const int c = h->sched_cfg.spin_split;
    if (h->noalloc_call || c < 0) return 0;
    if (c == 1 || c == 2) return c;
    return implicit ? 2 : 0;
}

int launch_spin_mult(hphi_ham *h, const MultArgs &m)
{
    const hphi_basis *b = h->basis;
    const Species &s = b->sp[0];
    if (!spin_stored_path(h)) {
        if (m.raw_out && m.nvec * dtype_lanes(m.dtype) == 1)
            return fail(HPHI_ERR_UNSUPPORTED, "raw product output of one real vector needs the stored-list spin kernel");
        return launch_spin_mult_implicit(h, m);
    }
    SpinKArgs a{};
    a.states = s.d_states.as<uint32_t>();
    a.dim = s.dim;
    a.bonds = h->d_bonds.as<SpinBondDev>();
    a.nb = h->n_bonds;
    a.hz = h->has_field ? h->d_hz.as<double>() : nullptr;
    a.n_sites = b->n_sites;
    a.lo_rank = s.d_lo_rank.as<uint32_t>();
    a.hi_off = s.d_hi_off32.as<uint32_t>();
    a.n_lo = s.n_lo;
    a.n_hi = s.n_hi;
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.coef = m.coef;
    a.nd = m.dots;
    a.dot_raw = m.dot_raw;
    a.red = m.red;
    a.coef_cplx = m.coef_cplx;
    a.raw_out = m.raw_out;
    a.cocg = static_cast<CgDev *>(m.cocg);
    const int nv = m.nvec * dtype_lanes(m.dtype);
    size_t tab = sizeof(uint32_t) * ((size_t(1) << s.n_lo) + (size_t(1) << s.n_hi));
    // the same tables with lo_rank in 16 bits (its values are ranks among
    // the same-popcount low patterns: below 65536 for up to 18 low sites)
    const size_t tab_c = sizeof(uint32_t) * (size_t(1) << s.n_hi) + sizeof(uint16_t) * (size_t(1) << s.n_lo);
    // (up to 128 bytes per state, 32 with fused dots: wider accumulators
    // do not fit the registers of a 1024-thread workgroup)
    const size_t state_bytes = (size_t)m.nvec * dtype_lanes(m.dtype) * (dtype_is_f32(m.dtype) ? 4 : 8);
    // 32-bit tables in LDS while they leave room for 2048 threads per CU;
    // beyond that the narrowed tables with 1024-thread workgroups (two per
    // CU where they fit: 23-24 sites)
    const int per_cu_sched = h->sched_cfg.spin_per_cu;
    const int per_cu_1 = std::min(per_cu_sched, std::max(1, (int)((160 * 1024) / (tab + 4096))));
    const bool narrow_ok = tab_c <= 96 * 1024 && s.n_lo <= 18 && state_bytes <= (m.dots ? 32u : 128u);
    int lds = (tab <= 96 * 1024 && (per_cu_1 * kBlock >= 2 * kSpinBigBlock || !narrow_ok)) ? 1 : narrow_ok ? 2 : 0;
    switch (h->sched_cfg.spin_tables) {
    case 1:
        if (tab > 96 * 1024) return fail(HPHI_ERR_UNSUPPORTED, "spin_tables 1: %zu bytes of tables exceed LDS", tab);
        lds = 1;
        break;
    case 2:
        if (!narrow_ok) return fail(HPHI_ERR_UNSUPPORTED, "spin_tables 2: narrowed tables do not fit this product");
        lds = 2;
        break;
    case 3: lds = 0; break;
    default: break;
    }
    if (lds == 2) tab = tab_c;
    const int bs = lds == 2 ? kSpinBigBlock : kBlock;
    int64_t need = (s.dim + bs - 1) / bs;
    // workgroups per CU from the schedule, capped by the LDS the tables use
    // (and by the static reduction scratch of a 1024-thread workgroup)
    int per_cu = per_cu_sched;
    if (lds == 1) per_cu = per_cu_1;
    if (lds == 2) per_cu = std::min(2, std::max(1, (int)((160 * 1024) / (tab + 9 * 1024))));
    int64_t cap = (int64_t)(h->basis->ctx->n_cu > 0 ? h->basis->ctx->n_cu : 256) * per_cu;
    if (cap > kMaxGrid) cap = kMaxGrid;
    int grid = (int)(need < cap ? need : cap);
    if (grid < 1) grid = 1;
    // split product: the bonds with an end in the low half into w, then
    // the high-half bonds and the caller's epilogue in slab order
    const int mode = spin_split_mode(h, false);
    bool split = mode != 0 && !m.dots && !m.cocg && m.v != m.w && (!m.u || m.u != m.w) &&
                 (!m.acc || m.acc != m.w) && (!m.raw_out || m.raw_out != m.w);
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
        a.coef_cplx = 0;
        a.raw_out = nullptr;
        a.nd = 0;
        a.cocg = nullptr;
        if (dtype_is_f32(m.dtype)) HPHI_TRY(launch_spin_nv<float>(nv, a, lds, grid, tab, m.stream));
        else HPHI_TRY(launch_spin_nv<double>(nv, a, lds, grid, tab, m.stream));
        return launch_spin_hi_pass(h, m);
    }
    if (dtype_is_f32(m.dtype)) return launch_spin_nv<float>(nv, a, lds, grid, tab, m.stream);
    return launch_spin_nv<double>(nv, a, lds, grid, tab, m.stream);
}

} // namespace hphi

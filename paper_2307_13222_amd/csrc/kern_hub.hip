// Hubbard H*v (HPhi update paper Sec. 3.4, Eq. Hquench with static U;
// Sec. 5): H = -sum t (c+c + h.c.) + sum_i U_i n_i,up n_i,dn.
//
// The (N_up, N_dn) sector is the product of two one-species bases, and with
// up-major indices a vector is the matrix V[r_up][r_dn]. Because a hop acts
// on one species only, H is the Kronecker sum
//   W = T_up V + V T_dn^T + U D o V,   D[r_up][r_dn] = (#doubly occupied sites),
// where T_sigma is the one-species hopping matrix with the fermion sign
// (-1)^(occupied same-species sites strictly between i and j) (all up
// orbitals ordered before all down orbitals). The two terms want different
// tilings, so the product runs as two kernels:
//   k_hub_rows: one workgroup per row r_up; the row V[r_up][:] is staged in
//               LDS, then W[r_up][c] = D o V + sum_{c'} T_dn[c][c'] V[r_up][c']
//               gathers from LDS. The down lists are sliced ELL (chunks of
//               64 columns, entry-major), so a wave's table loads coalesce;
//   k_hub_cols: XCD-aware column slabs: each XCD sweeps all rows of one slab
//               of CW columns at a time, so V[:, slab] stays in that XCD's L2
//               while W[r][slab] += sum_{r'} T_up[r][r'] V[r'][slab] reads
//               whole cache lines of the slab; the Lanczos/TPQ epilogue and
//               the FP64 partial dots are fused here.
// Table entries: target rank | value class << 24 | sign << 31.
#include "kern_common.h"

namespace hphi {

struct HubKArgs {
    const uint32_t *ups, *dns;
    int64_t dup, ddn;
    const uint32_t *off_up, *nbr_up;
    const uint32_t *sell_base_dn, *sell_width_dn, *sell_dn;
    const double *coef;    // value class -> -t (class 127 = 0)
    const double *u_site;
    int n_sites;
    int uniform_u;
    double u0;
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    const double *ecoef;   // epilogue [c1, c2]
    int nd;
    int dot_raw;
    Reduce red;
    int nslab, groups;     // column kernel geometry
};

template <typename S>
__device__ __forceinline__ S hub_diag(const HubKArgs &a, uint32_t u, uint32_t d)
{
    uint32_t both = u & d;
    if (a.uniform_u) return (S)(a.u0 * (double)__builtin_popcount(both));
    S s = (S)0;
    while (both) {
        int i = __builtin_ctz(both);
        s += (S)a.u_site[i];
        both &= both - 1u;
    }
    return s;
}

template <typename S>
__device__ __forceinline__ S entry_val(uint32_t e, const S *coef)
{
    S c = coef[(e >> 24) & 127u];
    return (e >> 31) ? -c : c;
}

// ---------------------------------------------------------------- rows --
// One workgroup per r_up (grid-stride). NV = 1 (real) or 2 (complex).
// Thread t handles columns t, t + blockDim, ...: a wave covers one aligned
// 64-column chunk of the sliced-ELL table.
template <typename S, int NV, bool LDS_ROW>
__global__ __launch_bounds__(1024) void k_hub_rows(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    S *s_coef = reinterpret_cast<S *>(smem_raw);
    S *s_row = s_coef + 128;
    for (int i = threadIdx.x; i < 128; i += blockDim.x) s_coef[i] = (S)a.coef[i];
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const int64_t ddn = a.ddn;
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * ddn * NV;
        __syncthreads();
        if constexpr (LDS_ROW) {
            for (int64_t i = threadIdx.x; i < ddn * NV; i += blockDim.x) s_row[i] = vrow[i];
            __syncthreads();
        }
        const S *row = LDS_ROW ? s_row : vrow;
        const uint32_t uu = a.ups[ru];
        for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) {
            const uint32_t d = a.dns[c];
            const S dg = hub_diag<S>(a, uu, d);
            S acc[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] = dg * row[c * NV + j];
            const int64_t ch = c >> 6;
            const uint32_t *ent = a.sell_dn + a.sell_base_dn[ch] + (c & 63);
            const uint32_t width = a.sell_width_dn[ch];
            for (uint32_t k = 0; k < width; ++k) {
                const uint32_t e = ent[(size_t)k * 64];
                const S val = entry_val<S>(e, s_coef);
                const uint32_t col = e & kNbrColMask;
#pragma unroll
                for (int j = 0; j < NV; ++j) acc[j] += val * row[(size_t)col * NV + j];
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) w[((size_t)ru * ddn + c) * NV + j] = acc[j];
        }
    }
}

// ---------------------------------------------------------------- cols --
// Persistent grid of 8 * groups workgroups. Workgroups are dispatched to
// the XCDs round-robin, so workgroup b runs on XCD b % 8; XCD x walks the
// slabs x, x + 8, x + 16, ... and its `groups` workgroups split each slab's
// rows, moving through the slabs together: the XCD's L2 holds V[:, slab].
template <typename S, int NV, int CW, bool DOTS>
__global__ __launch_bounds__(256) void k_hub_cols(HubKArgs a)
{
    __shared__ S s_coef[128];
    __shared__ double sh_red[16];
    __shared__ double sh_blk[4];
    for (int i = threadIdx.x; i < 128; i += blockDim.x) s_coef[i] = (S)a.coef[i];
    __syncthreads();
    const int bid = blockIdx.x;
    const int xcd = bid & 7, g = bid >> 3;
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *__restrict__ accp = static_cast<S *>(a.acc_out);
    double c1 = 1.0, c2 = 0.0;
    if (a.ecoef) {
        c1 = a.ecoef[0];
        c2 = a.ecoef[1];
    }
    const S c1s = (S)c1, c2s = (S)c2;
    double d0[NV], d1[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) d0[j] = d1[j] = 0.0;

    const int64_t ddn = a.ddn, dup = a.dup;
    const int64_t rows_per_g = (dup + a.groups - 1) / a.groups;
    const int64_t r0 = (int64_t)g * rows_per_g;
    const int64_t r1 = r0 + rows_per_g < dup ? r0 + rows_per_g : dup;
    constexpr int RPW = 64 / CW;              // rows per wave pass
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int slab = xcd; slab < a.nslab; slab += 8) {
        const int64_t col = (int64_t)slab * CW + (lane % CW);
        const bool colok = col < ddn;
        for (int64_t r = r0 + wid * RPW + lane / CW; r < r1; r += 4 * RPW) {
            if (!colok) continue;
            const size_t me = (size_t)r * ddn + col;
            S acc[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] = w[me * NV + j];
            const uint32_t e0 = a.off_up[r], e1 = a.off_up[r + 1];
            for (uint32_t e = e0; e < e1; ++e) {
                const uint32_t ent = a.nbr_up[e];
                const S val = entry_val<S>(ent, s_coef);
                const size_t src = (size_t)(ent & kNbrColMask) * ddn + col;
#pragma unroll
                for (int j = 0; j < NV; ++j) acc[j] += val * v[src * NV + j];
            }
            S out[NV], raw[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                raw[j] = acc[j];
                out[j] = c1s * acc[j];
            }
            if (u) {
#pragma unroll
                for (int j = 0; j < NV; ++j) out[j] += c2s * u[me * NV + j];
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) w[me * NV + j] = out[j];
            if (accp) {
#pragma unroll
                for (int j = 0; j < NV; ++j) accp[me * NV + j] += out[j];
            }
            if constexpr (DOTS) {
#pragma unroll
                for (int j = 0; j < NV; ++j) {
                    const double o = a.dot_raw ? (double)raw[j] : (double)out[j];
                    d0[j] += (double)v[me * NV + j] * o;
                    d1[j] += o * o;
                }
            }
        }
    }
    if constexpr (DOTS) {
        double vals[2 * NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            vals[j] = d0[j];
            vals[NV + j] = d1[j];
        }
        block_sum<2 * NV>(vals, sh_red);
        if (threadIdx.x == 0)
            for (int j = 0; j < 2 * NV; ++j) sh_blk[j] = vals[j];
        __syncthreads();
        grid_finish(sh_blk, 2 * NV, a.red, sh_red);
    }
}

// Column-slab geometry: CW columns per slab, G workgroups per slab. The
// defaults keep one 16-column slab (dim_up * 128 B for FP64) per XCD L2 with
// about one slab's worth of workgroups resident per XCD.
struct HubGeom {
    int cw = 16;
    int groups = 256;
};
static HubGeom g_hub_geom;

extern "C" int hphi_internal_set_hub_geom(int cw, int groups)
{
    if (!(cw == 16 || cw == 32 || cw == 64) || groups < 1 || groups > 4096) return HPHI_ERR_INVALID_ARG;
    g_hub_geom.cw = cw;
    g_hub_geom.groups = groups;
    return HPHI_OK;
}

template <typename S, int NV, int CW>
static void launch_cols_t(const HubKArgs &a, int grid, hipStream_t st)
{
    if (a.nd) hipLaunchKernelGGL((k_hub_cols<S, NV, CW, true>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_hub_cols<S, NV, CW, false>), dim3(grid), dim3(256), 0, st, a);
}

template <typename S, int NV>
static int launch_hub_t(hphi_ham *h, HubKArgs a, hipStream_t st)
{
    const int ncu = h->basis->ctx->n_cu > 0 ? h->basis->ctx->n_cu : 256;
    // rows kernel
    size_t row_bytes = (size_t)a.ddn * NV * sizeof(S) + 128 * sizeof(S);
    bool lds_row = row_bytes <= 160 * 1024;
    int per_cu = lds_row ? (int)((160 * 1024) / row_bytes) : 4;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    int64_t grid_r = (int64_t)ncu * per_cu;
    if (grid_r > a.dup) grid_r = a.dup;
    int threads = 1024;
    if (lds_row) {
        hipFuncSetAttribute((const void *)k_hub_rows<S, NV, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)row_bytes);
        hipLaunchKernelGGL((k_hub_rows<S, NV, true>), dim3((unsigned)grid_r), dim3(threads),
                           row_bytes, st, a);
    } else {
        hipLaunchKernelGGL((k_hub_rows<S, NV, false>), dim3((unsigned)grid_r), dim3(threads),
                           128 * sizeof(S), st, a);
    }
    HPHI_HIP(hipGetLastError());
    // column kernel
    const int cw = g_hub_geom.cw;
    int groups = g_hub_geom.groups;
    const int64_t min_rows_per_group = 4 * (64 / cw);
    if ((int64_t)groups * min_rows_per_group > a.dup)
        groups = (int)std::max<int64_t>(1, a.dup / min_rows_per_group);
    a.groups = groups;
    a.nslab = (int)((a.ddn + cw - 1) / cw);
    const int64_t grid_c = 8 * (int64_t)groups;
    if (grid_c * 2 * NV > (int64_t)kMaxGrid * 64)
        return fail(HPHI_ERR_UNSUPPORTED, "Hubbard column grid beyond the reduction scratch");
    switch (cw) {
    case 16: launch_cols_t<S, NV, 16>(a, (int)grid_c, st); break;
    case 32: launch_cols_t<S, NV, 32>(a, (int)grid_c, st); break;
    default: launch_cols_t<S, NV, 64>(a, (int)grid_c, st); break;
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_hub_mult(hphi_ham *h, const MultArgs &m)
{
    const hphi_basis *b = h->basis;
    HubKArgs a{};
    a.ups = b->sp[0].d_states.as<uint32_t>();
    a.dns = b->sp[1].d_states.as<uint32_t>();
    a.dup = b->sp[0].dim;
    a.ddn = b->sp[1].dim;
    a.off_up = h->hub.off[0].as<uint32_t>();
    a.nbr_up = h->hub.nbr[0].as<uint32_t>();
    a.sell_base_dn = h->hub.sell_base[1].as<uint32_t>();
    a.sell_width_dn = h->hub.sell_width[1].as<uint32_t>();
    a.sell_dn = h->hub.sell[1].as<uint32_t>();
    a.coef = h->hub.coef.as<double>();
    a.u_site = h->hub.u_site.as<double>();
    a.n_sites = b->n_sites;
    a.uniform_u = h->hub.uniform_u ? 1 : 0;
    a.u0 = h->hub.u0;
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.ecoef = m.coef;
    a.nd = m.dots;
    a.dot_raw = m.dot_raw;
    a.red = m.red;
    const int nv = m.nvec * dtype_lanes(m.dtype);
    const bool f32 = dtype_is_f32(m.dtype);
    if (nv == 1) return f32 ? launch_hub_t<float, 1>(h, a, m.stream) : launch_hub_t<double, 1>(h, a, m.stream);
    if (nv == 2) return f32 ? launch_hub_t<float, 2>(h, a, m.stream) : launch_hub_t<double, 2>(h, a, m.stream);
    return fail(HPHI_ERR_UNSUPPORTED, "Hubbard H*v supports one real or one complex vector per call");
}

} // namespace hphi

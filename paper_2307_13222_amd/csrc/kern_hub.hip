// Hubbard H*v (HPhi update paper Sec. 3.4, Eq. Hquench with static U;
// Sec. 5): H = -sum t (c+c + h.c.) + sum_i U_i n_i,up n_i,dn (the two-body
// terms of Eq. ham_general, where present, are added by k_hub_pairs
// between the two kernels below).
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

constexpr int kColsRows = 128;          // most rows per work item of the column kernel
constexpr int kColsLdsEntries = 4096;   // staged neighbour entries per item (>= rows * max degree)

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
    int item_rows;         // rows per work item (<= kColsRows)
    int row_cols;          // columns per lane of the T_up queue kernel (1, 2)
    unsigned *sched;       // 8 per-XCD item queues + completion counter
    // uniform |t| fast path
    const uint32_t *fs_base, *fs_wp, *fs_wm;
    const uint16_t *fs_ent;
    const uint32_t *fu_off, *fu_mid, *fu_ent;
    const uint32_t *fb_base, *fb_w;
    const uint32_t *fb_ent;
    const uint32_t *fc_ent;   // pre-scaled slot words for this element size (or null)
    double t0;
    const double *coef_im;   // imaginary parts of the class values (complex transfers; null: real)
    int coef_cplx;
    int hb;                // column kernel: batched list walk, one wave per row
    // Lanczos update fused into the rows kernel (null lz_q: none)
    LzDev *lz;
    double *lz_alpha, *lz_beta;
    const void *lz_q;      // q_{k-1}: v <- v - f q_{k-1} before the product
    Reduce lz_red;
    const uint32_t *row_of;   // column kernels: row processed at position p (null: p)
    hipEvent_t ev_mid;        // recorded between the rows and the column kernel (null: none)
    // T_up tile kernel (k_hub_up_tile): blocks of up rows, per-position lists
    const uint32_t *ft_blk, *ft_pos, *ft_off, *ft_cnt, *ft_ent;
    int ft_nb;
    uint32_t ft_tile_bytes;   // LDS bytes of the staged block (most rows x row stride)
    // row pitch (elements) of v, w, u and lz_q: ddn for caller vectors; the
    // Lanczos run pads rows to whole cache lines for the rows kernels
    // k_hub_rows_fp / k_hub_rows_fz and the tile kernel
    int64_t ld;
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
// 64-column chunk of the sliced-ELL table. CPLX (NV = 2): complex class
// values (c_re + i c_im) times the complex vector.
template <typename S, int NV, bool LDS_ROW, bool CPLX = false>
__global__ __launch_bounds__(1024) void k_hub_rows(HubKArgs a)
{
    static_assert(!CPLX || NV == 2, "complex coefficients need complex vectors");
    extern __shared__ unsigned char smem_raw[];
    S *s_coef = reinterpret_cast<S *>(smem_raw);
    S *s_coef_im = s_coef + 128;
    S *s_row = s_coef + (CPLX ? 256 : 128);
    for (int i = threadIdx.x; i < 128; i += blockDim.x) {
        s_coef[i] = (S)a.coef[i];
        if constexpr (CPLX) s_coef_im[i] = (S)a.coef_im[i];
    }
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
            uint32_t k = 0;
            // sixteen table loads in flight per lane, then the LDS gathers
            for (; k + 16 <= width; k += 16) {
                uint32_t e[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) e[t] = ent[(size_t)(k + t) * 64];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const S val = entry_val<S>(e[t], s_coef);
                    const uint32_t col = e[t] & kNbrColMask;
                    if constexpr (CPLX) {
                        const S vi = entry_val<S>(e[t], s_coef_im);
                        const S x0 = row[(size_t)col * 2], x1 = row[(size_t)col * 2 + 1];
                        acc[0] += val * x0 - vi * x1;
                        acc[1] += val * x1 + vi * x0;
                    } else {
#pragma unroll
                        for (int j = 0; j < NV; ++j) acc[j] += val * row[(size_t)col * NV + j];
                    }
                }
            }
            for (; k < width; ++k) {
                const uint32_t e = ent[(size_t)k * 64];
                const S val = entry_val<S>(e, s_coef);
                const uint32_t col = e & kNbrColMask;
                if constexpr (CPLX) {
                    const S vi = entry_val<S>(e, s_coef_im);
                    const S x0 = row[(size_t)col * 2], x1 = row[(size_t)col * 2 + 1];
                    acc[0] += val * x0 - vi * x1;
                    acc[1] += val * x1 + vi * x0;
                } else {
#pragma unroll
                    for (int j = 0; j < NV; ++j) acc[j] += val * row[(size_t)col * NV + j];
                }
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) __builtin_nontemporal_store(acc[j], &w[((size_t)ru * ddn + c) * NV + j]);
        }
    }
}

// Complex class values (complex transfers) on complex vectors whose whole
// row exceeds LDS: the row is staged one lane at a time. With class values
// A + iB, the re lane gives A x_re to the real part and B x_re to the
// imaginary part of W, the im lane A x_im to the imaginary and -B x_im to
// the real part: the re lane writes the row of W, the im lane adds to it
// (the row, 2 x ddn values, stays in L2 between the lanes).
template <typename S>
__global__ __launch_bounds__(1024) void k_hub_rows_cl(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    S *s_coef = reinterpret_cast<S *>(smem_raw);
    S *s_coef_im = s_coef + 128;
    S *s_row = s_coef + 256;
    for (int i = threadIdx.x; i < 128; i += blockDim.x) {
        s_coef[i] = (S)a.coef[i];
        s_coef_im[i] = (S)a.coef_im[i];
    }
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const int64_t ddn = a.ddn;
    const int T = blockDim.x, tid = threadIdx.x;
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * ddn * 2;
        S *wrow = w + (size_t)ru * ddn * 2;
        const uint32_t uu = a.ups[ru];
        for (int ln = 0; ln < 2; ++ln) {
            __syncthreads();   // the previous lane's (or row's) gathers have finished
            for (int64_t i = tid; i < ddn; i += T) s_row[i] = vrow[2 * i + ln];
            __syncthreads();
            for (int64_t c = tid; c < ddn; c += T) {
                const int64_t ch = c >> 6;
                const uint32_t *ent = a.sell_dn + a.sell_base_dn[ch] + (c & 63);
                const uint32_t width = a.sell_width_dn[ch];
                S sa = (S)0, sb = (S)0;
                uint32_t k = 0;
                // eight table loads in flight, then the LDS gathers
                for (; k + 8 <= width; k += 8) {
                    uint32_t en[8];
#pragma unroll
                    for (int t = 0; t < 8; ++t) en[t] = ent[(size_t)(k + t) * 64];
#pragma unroll
                    for (int t = 0; t < 8; ++t) {
                        const S x = s_row[en[t] & kNbrColMask];
                        sa += entry_val<S>(en[t], s_coef) * x;
                        sb += entry_val<S>(en[t], s_coef_im) * x;
                    }
                }
                for (; k < width; ++k) {
                    const uint32_t en = ent[(size_t)k * 64];
                    const S x = s_row[en & kNbrColMask];
                    sa += entry_val<S>(en, s_coef) * x;
                    sb += entry_val<S>(en, s_coef_im) * x;
                }
                const S dx = hub_diag<S>(a, uu, a.dns[c]) * s_row[c];
                if (ln == 0) {
                    wrow[2 * c] = dx + sa;
                    wrow[2 * c + 1] = sb;
                } else {
                    // the same thread wrote this element in the re lane
                    wrow[2 * c] = wrow[2 * c] - sb;
                    wrow[2 * c + 1] = wrow[2 * c + 1] + (dx + sa);
                }
            }
        }
    }
}

// ---------------------------------------------------------------- cols --
// Persistent grid. A work item is (slab, chunk of kColsRows rows); XCD x
// owns the slabs x, x + 8, x + 16, ... and hands out its items in slab
// order from its own atomic queue, so the workgroups resident on one XCD
// work on one or two slabs at a time and that XCD's L2 holds V[:, slab].
// A workgroup learns its XCD from the XCC_ID hardware register; when its
// queue is empty it takes items from the other XCDs' queues, so every item
// runs whatever the placement of workgroups on XCDs. w and u are streamed
// non-temporally so they do not displace the slab in L2.
// Dot partials are kept per item (item = slab * nchunk + chunk), so the
// final sum, taken in item order by the last workgroup to finish, does not
// depend on which workgroup ran which item: results are run-to-run
// identical. That workgroup also re-arms the queues.
__device__ __forceinline__ int xcc_id() { return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u); }

template <typename S, int NV, int CW, bool DOTS, bool CPLX = false>
__global__ __launch_bounds__(256) void k_hub_cols(HubKArgs a)
{
    static_assert(!CPLX || NV == 2, "complex coefficients need complex vectors");
    __shared__ S s_coef[128];
    __shared__ S s_coef_im[CPLX ? 128 : 1];
    __shared__ double sh_red[4 * 2 * NV + 8];
    __shared__ uint32_t s_ent[kColsLdsEntries];
    __shared__ uint32_t s_off[kColsRows + 1];
    __shared__ int s_item;
    __shared__ unsigned s_last;
    for (int i = threadIdx.x; i < 128; i += blockDim.x) {
        s_coef[i] = (S)a.coef[i];
        if constexpr (CPLX) s_coef_im[i] = (S)a.coef_im[i];
    }
    const int home = xcc_id();
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

    const int64_t ddn = a.ddn, dup = a.dup;
    const int nchunk = (int)((dup + a.item_rows - 1) / a.item_rows);
    constexpr int RPW = 64 / CW;              // rows per wave pass
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int q = home, tries = 0;
    for (;;) {
        // next item: own XCD first, then the others in turn
        __syncthreads();
        if (threadIdx.x == 0) {
            int it = -1;
            while (tries < 8) {
                const int nsl_q = q < a.nslab ? (a.nslab - q + 7) / 8 : 0;
                const int cand = (int)atomicAdd(&a.sched[q], 1u);
                if (cand < nsl_q * nchunk) {
                    it = q + 8 * cand;   // (queue, index within the queue)
                    break;
                }
                q = (q + 1) & 7;
                ++tries;
            }
            s_item = it;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        const int iq = item & 7, idx = item >> 3;
        const int slab = iq + 8 * (idx / nchunk);
        const int chunk = idx % nchunk;
        const int64_t r0 = (int64_t)chunk * a.item_rows;
        const int64_t r1 = r0 + a.item_rows < dup ? r0 + a.item_rows : dup;
        // stage the chunk's neighbour lists
        {
            const uint32_t base = a.off_up[r0];
            for (int64_t i = threadIdx.x; i <= r1 - r0; i += blockDim.x) s_off[i] = a.off_up[r0 + i] - base;
            const uint32_t n = a.off_up[r1] - base;
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_ent[i] = a.nbr_up[base + i];
        }
        __syncthreads();
        double d0[NV], d1[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) d0[j] = d1[j] = 0.0;
        const int64_t col = (int64_t)slab * CW + (lane % CW);
        const bool colok = col < ddn;
        for (int64_t r = r0 + wid * RPW + lane / CW; r < r1; r += 4 * RPW) {
            if (!colok) continue;
            const size_t me = (size_t)r * ddn + col;
            S acc[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] = __builtin_nontemporal_load(&w[me * NV + j]);
            const uint32_t e1 = s_off[r - r0 + 1];
            uint32_t e = s_off[r - r0];
            // up to GB neighbour rows in flight at once, then the FMAs
            constexpr int GB = NV == 1 ? 32 : 16;
            for (; e < e1; e += GB) {
                S nv[GB][NV];
                S val[GB], vim[CPLX ? GB : 1];
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    const bool ok = e + t < e1;
                    const uint32_t ent = s_ent[ok ? e + t : e];
                    val[t] = ok ? entry_val<S>(ent, s_coef) : (S)0;
                    if constexpr (CPLX) vim[t] = ok ? entry_val<S>(ent, s_coef_im) : (S)0;
                    const size_t src = (size_t)(ent & kNbrColMask) * ddn + col;
#pragma unroll
                    for (int j = 0; j < NV; ++j) nv[t][j] = ok ? v[src * NV + j] : (S)0;
                }
#pragma unroll
                for (int t = 0; t < GB; ++t) {
                    if constexpr (CPLX) {
                        acc[0] += val[t] * nv[t][0] - vim[t] * nv[t][1];
                        acc[1] += val[t] * nv[t][1] + vim[t] * nv[t][0];
                    } else {
#pragma unroll
                        for (int j = 0; j < NV; ++j) acc[j] += val[t] * nv[t][j];
                    }
                }
            }
            for (; e < e1; ++e) {
                const uint32_t ent = s_ent[e];
                const S val = entry_val<S>(ent, s_coef);
                const size_t src = (size_t)(ent & kNbrColMask) * ddn + col;
                if constexpr (CPLX) {
                    const S vi = entry_val<S>(ent, s_coef_im);
                    const S x0 = v[src * 2], x1 = v[src * 2 + 1];
                    acc[0] += val * x0 - vi * x1;
                    acc[1] += val * x1 + vi * x0;
                } else {
#pragma unroll
                    for (int j = 0; j < NV; ++j) acc[j] += val * v[src * NV + j];
                }
            }
            S out[NV], raw[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) raw[j] = acc[j];
            if (a.coef_cplx) {
                S uu[NV];
                if (u)
#pragma unroll
                    for (int j = 0; j < NV; ++j) uu[j] = __builtin_nontemporal_load(&u[me * NV + j]);
                epilogue<S, NV>(raw, u ? uu : nullptr, 1, a.ecoef, out);
            } else {
#pragma unroll
                for (int j = 0; j < NV; ++j) out[j] = c1s * acc[j];
                if (u) {
#pragma unroll
                    for (int j = 0; j < NV; ++j) out[j] += c2s * __builtin_nontemporal_load(&u[me * NV + j]);
                }
            }
#pragma unroll
            for (int j = 0; j < NV; ++j) __builtin_nontemporal_store(out[j], &w[me * NV + j]);
            if (accp) {
#pragma unroll
                for (int j = 0; j < NV; ++j)
                    __builtin_nontemporal_store(__builtin_nontemporal_load(&accp[me * NV + j]) + out[j],
                                                &accp[me * NV + j]);
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
        if constexpr (DOTS) {
            double vals[2 * NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) {
                vals[j] = d0[j];
                vals[NV + j] = d1[j];
            }
            block_sum<2 * NV>(vals, sh_red);
            if (threadIdx.x == 0) {
                const size_t slot = (size_t)slab * nchunk + chunk;
                for (int j = 0; j < 2 * NV; ++j) a.red.partial[slot * 2 * NV + j] = vals[j];
            }
        }
    }
    // last workgroup out: final dot sums in item order, re-arm the queues
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = (atomicAdd(&a.sched[8], 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if constexpr (DOTS) {
        const size_t nitems = (size_t)a.nslab * nchunk;
        for (int j = 0; j < 2 * NV; ++j) {
            double s = 0.0;
            for (size_t it = threadIdx.x; it < nitems; it += blockDim.x)
                s += __builtin_nontemporal_load(&a.red.partial[it * 2 * NV + j]);
            double vv[1] = {s};
            block_sum<1>(vv, sh_red);
            if (threadIdx.x == 0) a.red.result[j] = vv[0];
        }
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 8; ++i) a.sched[i] = 0u;
        a.sched[8] = 0u;
        __threadfence();
    }
}

// ------------------------------------------------- uniform |t| fast path --
// Every transfer has magnitude t0, so each list splits into the entries
// whose element is -t0 (plus) and +t0 (minus):
//   (T v)[x] = -t0 (sum_plus v - sum_minus v),
// one address operation, one load and one add per neighbour, no value or
// sign decoding. Rows kernel: uint16 column entries, padding points at a
// zero slot behind the staged row.
template <typename S, int NV>
__global__ __launch_bounds__(1024) void k_hub_rows_f(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    S *s_row = reinterpret_cast<S *>(smem_raw);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const int64_t ddn = a.ddn;
    const S nt0 = (S)(-a.t0);
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * ddn * NV;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < ddn * NV; i += blockDim.x) s_row[i] = vrow[i];
        if (threadIdx.x < NV) s_row[ddn * NV + threadIdx.x] = (S)0;
        __syncthreads();
        const uint32_t uu = a.ups[ru];
        for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) {
            const S dg = hub_diag<S>(a, uu, a.dns[c]);
            const int64_t ch = c >> 6;
            const uint16_t *ent = a.fs_ent + a.fs_base[ch] + (c & 63);
            const uint32_t wp = a.fs_wp[ch], wt = wp + a.fs_wm[ch];
            S ap[NV], am[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) ap[j] = am[j] = (S)0;
            uint32_t k = 0;
            for (; k + 8 <= wp; k += 8) {
                uint32_t e[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) e[t] = ent[(k + t) * 64];
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < NV; ++j) ap[j] += s_row[e[t] * NV + j];
            }
            for (; k < wp; ++k) {
                const uint32_t e = ent[k * 64];
#pragma unroll
                for (int j = 0; j < NV; ++j) ap[j] += s_row[e * NV + j];
            }
            for (; k + 8 <= wt; k += 8) {
                uint32_t e[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) e[t] = ent[(k + t) * 64];
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < NV; ++j) am[j] += s_row[e[t] * NV + j];
            }
            for (; k < wt; ++k) {
                const uint32_t e = ent[k * 64];
#pragma unroll
                for (int j = 0; j < NV; ++j) am[j] += s_row[e * NV + j];
            }
#pragma unroll
            for (int j = 0; j < NV; ++j)
                __builtin_nontemporal_store(dg * s_row[c * NV + j] + nt0 * (ap[j] - am[j]),
                                            &w[((size_t)ru * ddn + c) * NV + j]);
        }
    }
}

// LDS-resident column metadata: next to the staged row, the workgroup keeps
// every chunk's table offset and list widths and every column's down state
// (16 bits) for its whole persistent sweep over rows, so a column's table
// loads issue after one LDS read instead of a chain of L2 round trips.
// Each column's entries (up to 32, predicated) are requested at once.
template <typename S, int NV>
__global__ __launch_bounds__(1024) void k_hub_rows_fm(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int64_t ddn = a.ddn;
    const int64_t nch = (ddn + 63) >> 6;
    S *s_row = reinterpret_cast<S *>(smem_raw);
    uint32_t *s_base = reinterpret_cast<uint32_t *>(s_row + (ddn + 1) * NV);
    uint32_t *s_w = s_base + nch;
    uint16_t *s_d = reinterpret_cast<uint16_t *>(s_w + nch);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S nt0 = (S)(-a.t0);
    for (int64_t j = threadIdx.x; j < nch; j += blockDim.x) {
        s_base[j] = a.fs_base[j];
        s_w[j] = a.fs_wp[j] | ((a.fs_wp[j] + a.fs_wm[j]) << 16);
    }
    for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) s_d[c] = (uint16_t)a.dns[c];
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * ddn * NV;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < ddn * NV; i += blockDim.x) s_row[i] = vrow[i];
        if (threadIdx.x < NV) s_row[ddn * NV + threadIdx.x] = (S)0;
        __syncthreads();
        const uint32_t uu = a.ups[ru];
        for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) {
            // a wave's 64 columns are one chunk: its widths are wave-uniform
            const uint32_t mw = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_w[c >> 6]);
            const uint32_t wp = mw & 0xFFFFu, wt = mw >> 16;
            const uint16_t *ent = a.fs_ent + s_base[c >> 6] + (uint32_t)(c & 63);
            S ap[NV], am[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) ap[j] = am[j] = (S)0;
            // plus slots [0, wp), then minus slots [wp, wt), in slot order
            uint32_t t = 0;
            for (; t + 8 <= wp; t += 8) {
                uint32_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = ent[(t + k) * 64];
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int j = 0; j < NV; ++j) ap[j] += s_row[e[k] * NV + j];
            }
            for (; t < wp; ++t) {
                const uint32_t et = ent[t * 64];
#pragma unroll
                for (int j = 0; j < NV; ++j) ap[j] += s_row[et * NV + j];
            }
            for (; t + 8 <= wt; t += 8) {
                uint32_t e[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) e[k] = ent[(t + k) * 64];
#pragma unroll
                for (int k = 0; k < 8; ++k)
#pragma unroll
                    for (int j = 0; j < NV; ++j) am[j] += s_row[e[k] * NV + j];
            }
            for (; t < wt; ++t) {
                const uint32_t et = ent[t * 64];
#pragma unroll
                for (int j = 0; j < NV; ++j) am[j] += s_row[et * NV + j];
            }
            const S dg = hub_diag<S>(a, uu, (uint32_t)s_d[c]);
#pragma unroll
            for (int j = 0; j < NV; ++j)
                __builtin_nontemporal_store(dg * s_row[c * NV + j] + nt0 * (ap[j] - am[j]),
                                            &w[((size_t)ru * ddn + c) * NV + j]);
        }
    }
}

// Rows kernel with hop-ordered down slots: slot k of a 64-state chunk is one
// hop for all 64 lanes (a lane that the hop does not connect reads the zero
// slot). The lanes of a wave share their high-half pattern, so one slot's
// targets lie in one group of consecutive states of the row in LDS and the
// gathers rarely share a bank; two slots share a 32-bit word (15-bit
// columns, signs in bits 31 and 30, applied by flipping the sign bit). A
// lane's slots are consecutive in memory: up to 32 of them arrive in four
// 16-byte loads, issued for the next column while the current one gathers.
// Row metadata (chunk bases, widths, down states) is staged in LDS as in
// k_hub_rows_fm. Sum order: hops in input order.
// x with its sign flipped when bit 31 of s31 is set (the other bits of s31
// are zero).
__device__ __forceinline__ double flip_sign(double x, uint32_t s31)
{
    return __longlong_as_double(__double_as_longlong(x) ^ ((long long)s31 << 32));
}
__device__ __forceinline__ float flip_sign(float x, uint32_t s31)
{
    return __int_as_float(__float_as_int(x) ^ (int)s31);
}

template <typename S, int NV>
__device__ __forceinline__ void fb_gather(const uint4 (&q)[4], uint32_t nq, const S *s_row, S (&acc)[NV])
{
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if ((uint32_t)g >= nq) break;
        const uint32_t wd[4] = {q[g].x, q[g].y, q[g].z, q[g].w};
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const uint32_t wv = wd[p];
            const uint32_t c0 = wv & 0x7FFFu, c1 = (wv >> 15) & 0x7FFFu;
            const uint32_t s0 = wv & 0x80000000u, s1 = (wv << 1) & 0x80000000u;
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] += flip_sign(s_row[c0 * NV + j], s0);
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] += flip_sign(s_row[c1 * NV + j], s1);
        }
    }
}

// The same slots as fb_gather (one real vector) from pre-scaled words:
// bits 0..16 hold the low slot's LDS byte offset (element size times its
// column) with its sign in bit 0, bits 17..30 the high slot's column and
// bit 31 its sign. The row must sit at LDS address 0 (dynamic LDS of a
// kernel without static LDS; the launcher checks), so the offsets are LDS
// addresses as they are. Same sums in the same order as fb_gather:
// bit-identical results.
template <typename S>
__device__ __forceinline__ void fc_gather(const uint4 (&q)[4], uint32_t nq, S &acc)
{
    using lds_ptr = const __attribute__((address_space(3))) S *;
    constexpr bool F64 = sizeof(S) == 8;
    constexpr uint32_t lo_mask = F64 ? 0x1FFF8u : 0xFFFCu;
    constexpr uint32_t hi_shift = F64 ? 14u : 15u;
    constexpr uint32_t hi_mask = F64 ? 0x1FFF8u : 0xFFFCu;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        if ((uint32_t)g >= nq) break;
        const uint32_t wd[4] = {q[g].x, q[g].y, q[g].z, q[g].w};
        // the eight reads of a group first (all in flight), then the sums
        S x[8];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            x[2 * p] = *(lds_ptr)(wd[p] & lo_mask);
            x[2 * p + 1] = *(lds_ptr)((wd[p] >> hi_shift) & hi_mask);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            acc += flip_sign(x[2 * p], wd[p] << 31);
            acc += flip_sign(x[2 * p + 1], wd[p] & 0x80000000u);
        }
    }
}

template <typename S, int NV>
__global__ __launch_bounds__(1024) void k_hub_rows_fb(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int64_t ddn = a.ddn;
    const int64_t nch = (ddn + 63) >> 6;
    S *s_row = reinterpret_cast<S *>(smem_raw);
    uint32_t *s_base = reinterpret_cast<uint32_t *>(s_row + (ddn + 1) * NV);
    uint32_t *s_w = s_base + nch;
    uint16_t *s_d = reinterpret_cast<uint16_t *>(s_w + nch);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S nt0 = (S)(-a.t0);
    for (int64_t j = threadIdx.x; j < nch; j += blockDim.x) {
        s_base[j] = a.fb_base[j];
        s_w[j] = a.fb_w[j];
    }
    for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) s_d[c] = (uint16_t)a.dns[c];
    __syncthreads();
    // entries of column c: 16-byte words at fb_ent + base(c) + lane * width / 2
    auto load_col = [&](int64_t c, uint4 (&q)[4], uint32_t &nq) {
        nq = 0;
        if (c >= ddn) return;
        const uint32_t wc = s_w[c >> 6];
        nq = wc >> 3;
        const uint4 *p = reinterpret_cast<const uint4 *>(a.fb_ent + s_base[c >> 6] + (uint32_t)(c & 63) * (wc >> 1));
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if ((uint32_t)g < nq) q[g] = p[g];
    };
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * ddn * NV;
        __syncthreads();
        for (int64_t i = threadIdx.x; i < ddn * NV; i += blockDim.x) s_row[i] = vrow[i];
        if (threadIdx.x < NV) s_row[ddn * NV + threadIdx.x] = (S)0;
        uint4 cur[4], nxt[4];
        uint32_t ncur, nnxt;
        load_col(threadIdx.x, cur, ncur);
        __syncthreads();
        const uint32_t uu = a.ups[ru];
        for (int64_t c = threadIdx.x; c < ddn; c += blockDim.x) {
            load_col(c + blockDim.x, nxt, nnxt);
            S acc[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] = (S)0;
            fb_gather<S, NV>(cur, ncur, s_row, acc);
            const S dg = hub_diag<S>(a, uu, (uint32_t)s_d[c]);
#pragma unroll
            for (int j = 0; j < NV; ++j)
                __builtin_nontemporal_store(dg * s_row[c * NV + j] + nt0 * acc[j],
                                            &w[((size_t)ru * a.ld + c) * NV + j]);
#pragma unroll
            for (int g = 0; g < 4; ++g) cur[g] = nxt[g];
            ncur = nnxt;
        }
    }
}

// k_hub_rows_fb with the row staged by one batch of loads: each lane issues
// all of its (up to MAXE) loads of the row before the first LDS write, so a
// row costs one memory latency instead of one per element; the loads of row
// ru are issued before the barrier that waits for the gathers of the
// previous row. Needs ddn * NV <= MAXE * blockDim.x. Same slots, sums and
// summation order as k_hub_rows_fb: bit-identical results.
// FC: pre-scaled slot words (one real vector), see fc_gather.
template <typename S, int NV, int MAXE, bool FC = false>
__global__ __launch_bounds__(1024) void k_hub_rows_fp(HubKArgs a)
{
    static_assert(!FC || NV == 1, "pre-scaled slots address one real lane");
    const uint32_t *__restrict__ ent = FC ? a.fc_ent : a.fb_ent;
    extern __shared__ unsigned char smem_raw[];
    const int64_t ddn = a.ddn;
    const int64_t nch = (ddn + 63) >> 6;
    S *s_row = reinterpret_cast<S *>(smem_raw);
    uint32_t *s_base = reinterpret_cast<uint32_t *>(s_row + (ddn + 1) * NV);
    uint32_t *s_w = s_base + nch;
    uint16_t *s_d = reinterpret_cast<uint16_t *>(s_w + nch);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S nt0 = (S)(-a.t0);
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t nrow = (uint32_t)(ddn * NV);
    for (int64_t j = tid; j < nch; j += T) {
        s_base[j] = a.fb_base[j];
        s_w[j] = a.fb_w[j];
    }
    for (int64_t c = tid; c < ddn; c += T) s_d[c] = (uint16_t)a.dns[c];
    if (tid < NV) s_row[nrow + tid] = (S)0;
    // the 64 columns of a wave form one chunk (T is a multiple of 64), so
    // the chunk index, width and base are wave-uniform (scalar); lanes past
    // the row in the last chunk read its padding slots (in bounds, never
    // stored)
    auto load_col = [&](int64_t c, uint4 (&q)[4], uint32_t &nq) {
        const uint32_t k = __builtin_amdgcn_readfirstlane((uint32_t)(c >> 6));
        nq = 0;
        if (k >= (uint32_t)nch) return;
        const uint32_t wc = __builtin_amdgcn_readfirstlane(s_w[k]);
        const uint32_t base = __builtin_amdgcn_readfirstlane(s_base[k]);
        nq = wc >> 3;
        const uint4 *p = reinterpret_cast<const uint4 *>(ent + base + __umul24((uint32_t)(c & 63), wc >> 1));
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if ((uint32_t)g < nq) q[g] = p[g];
    };
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const S *vrow = v + (size_t)ru * a.ld * NV;
        // unconditional loads (indices past the row re-read its last
        // element) so that all of them are in flight together
        S tmp[MAXE];
#pragma unroll
        for (int e = 0; e < MAXE; ++e) {
            const uint32_t i = (uint32_t)e * T + tid;
            tmp[e] = vrow[i < nrow ? i : nrow - 1];
        }
        __syncthreads();    // every gather of the previous row has finished
#pragma unroll
        for (int e = 0; e < MAXE; ++e) {
            const uint32_t i = (uint32_t)e * T + tid;
            if (i < nrow) s_row[i] = tmp[e];
        }
        uint4 cur[4], nxt[4];
        uint32_t ncur, nnxt;
        load_col(tid, cur, ncur);
        __syncthreads();
        const uint32_t uu = a.ups[ru];
        for (int64_t c = tid; c < ddn; c += T) {
            load_col(c + T, nxt, nnxt);
            S acc[NV];
#pragma unroll
            for (int j = 0; j < NV; ++j) acc[j] = (S)0;
            if constexpr (FC)
                fc_gather<S>(cur, ncur, acc[0]);
            else
                fb_gather<S, NV>(cur, ncur, s_row, acc);
            const S dg = hub_diag<S>(a, uu, (uint32_t)s_d[c]);
#pragma unroll
            for (int j = 0; j < NV; ++j)
                __builtin_nontemporal_store(dg * s_row[c * NV + j] + nt0 * acc[j],
                                            &w[((size_t)ru * a.ld + c) * NV + j]);
#pragma unroll
            for (int g = 0; g < 4; ++g) cur[g] = nxt[g];
            ncur = nnxt;
        }
    }
}

// k_hub_rows_fp with the previous Lanczos step's update fused into the row
// staging (one real vector). The input v holds w_k, the unnormalized
// residual of the previous product; each element becomes
//   x = w_k - f q_{k-1},   f = alpha_{k-1} s_{k-1},  alpha_{k-1} = s_{k-1} <q_{k-1}, w_k>
// (the same expression, in the same precision, as the separate update
// kernel), is written back in place (it is q_k for the column kernel and the
// next step) and staged in LDS for this product. The last block to finish
// sums the blocks' |x|^2 in block order and performs the update's scalar
// step: alpha_{k-1}, beta_k = |x|, breakdown test, s_k = 1 / beta_k and the
// epilogue coefficients [s_k, -beta_k s_{k-1}] the column kernel then reads.
// Raw buffer loads: a wave-uniform resource (base, byte size) and a 32-bit
// per-lane byte offset, so that many loads in flight cost one address
// register each (the callers keep every offset inside the buffer).
constexpr int kBufWord3 = 0x00020000;   // gfx9-family buffer resource word 3
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, kBufWord3);
}
template <typename S> __device__ __forceinline__ S buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ __forceinline__ double buf_ld<double>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
template <> __device__ __forceinline__ float buf_ld<float>(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

// MAXE: row elements per lane (ddn <= MAXE * blockDim.x). All LDS is
// dynamic, the row first (at LDS address 0, as fc_gather needs) and the
// reduction scratch last; FC: pre-scaled slot words.
constexpr size_t kRowsFzTail = 160;   // reduction scratch after the row metadata
template <typename S, int MAXE, bool FC = false>
__global__ __launch_bounds__(1024) void k_hub_rows_fz(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int64_t ddn = a.ddn;
    const int64_t nch = (ddn + 63) >> 6;
    S *s_row = reinterpret_cast<S *>(smem_raw);
    uint32_t *s_base = reinterpret_cast<uint32_t *>(s_row + (ddn + 1));
    uint32_t *s_w = s_base + nch;
    uint16_t *s_d = reinterpret_cast<uint16_t *>(s_w + nch);
    // (byte offset from the LDS base, so the pointer stays an LDS pointer)
    const size_t red_off = ((size_t)(reinterpret_cast<unsigned char *>(s_d + ddn) - smem_raw) + 7) & ~(size_t)7;
    double *sh_red = reinterpret_cast<double *>(smem_raw + red_off);
    double *s_blk = sh_red + 16;
    unsigned *s_last = reinterpret_cast<unsigned *>(s_blk + 1);
    const uint32_t *__restrict__ ent = FC ? a.fc_ent : a.fb_ent;
    S *__restrict__ v = const_cast<S *>(static_cast<const S *>(a.v));
    const S *__restrict__ qp = static_cast<const S *>(a.lz_q);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S nt0 = (S)(-a.t0);
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t nrow = (uint32_t)ddn;
    LzDev *lz = a.lz;
    const bool corr = !lz->done;
    const double s_k1 = lz->s_cur;
    const double f = corr ? (s_k1 * lz->dot[0]) * s_k1 : 0.0;
    for (int64_t j = tid; j < nch; j += T) {
        s_base[j] = a.fb_base[j];
        s_w[j] = a.fb_w[j];
    }
    for (int64_t c = tid; c < ddn; c += T) s_d[c] = (uint16_t)a.dns[c];
    if (tid == 0) s_row[nrow] = (S)0;
    // the 64 columns of a wave form one chunk (T is a multiple of 64), so
    // the chunk index, width and base are wave-uniform (scalar); lanes past
    // the row in the last chunk read its padding slots (in bounds, never
    // stored)
    auto load_col = [&](int64_t c, uint4 (&q)[4], uint32_t &nq) {
        const uint32_t k = __builtin_amdgcn_readfirstlane((uint32_t)(c >> 6));
        nq = 0;
        if (k >= (uint32_t)nch) return;
        const uint32_t wc = __builtin_amdgcn_readfirstlane(s_w[k]);
        const uint32_t base = __builtin_amdgcn_readfirstlane(s_base[k]);
        nq = wc >> 3;
        const uint4 *p = reinterpret_cast<const uint4 *>(ent + base + __umul24((uint32_t)(c & 63), wc >> 1));
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if ((uint32_t)g < nq) q[g] = p[g];
    };
    double acc = 0.0;
    const uint32_t rbytes = nrow * (uint32_t)sizeof(S);
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        S *vrow = v + (size_t)ru * a.ld;
        const __amdgpu_buffer_rsrc_t rv = buf_rsrc(vrow, rbytes);
        const __amdgpu_buffer_rsrc_t rq = buf_rsrc(qp + (size_t)ru * a.ld, rbytes);
        // two rounds of loads (registers), each with all of its loads in
        // flight (indices past the row re-read its last element); the first
        // round is issued before the barrier that waits for the previous
        // row's gathers
        constexpr int E1 = (MAXE + 1) / 2;
#pragma unroll
        for (int hh = 0; hh < 2; ++hh) {
            const int e0 = hh ? E1 : 0, ne = hh ? MAXE - E1 : E1;
            S tv[E1], tq[E1];
#pragma unroll
            for (int e = 0; e < E1; ++e) {
                if (e >= ne) break;
                const uint32_t i = (uint32_t)(e0 + e) * T + tid;
                const uint32_t off = (i < nrow ? i : nrow - 1) * (uint32_t)sizeof(S);
                tv[e] = buf_ld<S>(rv, off);
                tq[e] = buf_ld<S>(rq, off);
            }
            if (hh == 0) __syncthreads();    // every gather of the previous row has finished
#pragma unroll
            for (int e = 0; e < E1; ++e) {
                if (e >= ne) break;
                const uint32_t i = (uint32_t)(e0 + e) * T + tid;
                if (i < nrow) {
                    const S x = corr ? (S)((double)tv[e] - f * (double)tq[e]) : tv[e];
                    s_row[i] = x;
                    if (corr) {
                        vrow[i] = x;
                        acc += (double)x * (double)x;
                    }
                }
            }
        }
        uint4 cur[4], nxt[4];
        uint32_t ncur, nnxt;
        load_col(tid, cur, ncur);
        __syncthreads();
        const uint32_t uu = a.ups[ru];
        for (int64_t c = tid; c < ddn; c += T) {
            load_col(c + T, nxt, nnxt);
            S accg[1] = {(S)0};
            if constexpr (FC)
                fc_gather<S>(cur, ncur, accg[0]);
            else
                fb_gather<S, 1>(cur, ncur, s_row, accg);
            const S dg = hub_diag<S>(a, uu, (uint32_t)s_d[c]);
            __builtin_nontemporal_store(dg * s_row[c] + nt0 * accg[0], &w[(size_t)ru * a.ld + c]);
#pragma unroll
            for (int g = 0; g < 4; ++g) cur[g] = nxt[g];
            ncur = nnxt;
        }
    }
    double vals[1] = {acc};
    block_sum<1>(vals, sh_red);
    if (tid == 0) s_blk[0] = vals[0];
    __syncthreads();
    if (grid_finish_at(s_blk, 1, a.lz_red, sh_red, s_last) && tid == 0 && corr) {
        const double b = sqrt(a.lz_red.result[0]);
        const double al = s_k1 * lz->dot[0];
        const int k = lz->iter;
        a.lz_alpha[k] = al;
        a.lz_beta[k + 1] = b;
        lz->iter = k + 1;
        if (!(b > 1e-13 * fmax(1.0, fabs(al)))) {
            lz->done = 1;
            lz->breakdown = 1;
        } else {
            lz->s_prev = s_k1;
            lz->s_cur = 1.0 / b;
            lz->coef[0] = lz->s_cur;
            lz->coef[1] = -b * s_k1;
        }
        __threadfence();
    }
}

// Rows kernel for NV > 1 interleaved lanes whose full row does not fit LDS
// (a complex FP64 row of the 4x4 sector is 206 KB): T_dn and U are real,
// so each lane of the row is a separate real row. Per row, lane by lane:
// stage the lane (stride NV; the row's cache lines stay in L2 between the
// lanes) in rounds of E loads per thread, gather its hop-ordered slots, and
// write the lane of W. Same slots, sums and order as k_hub_rows_fb per lane.
template <typename S, int NV, int E>
__global__ __launch_bounds__(1024) void k_hub_rows_fl(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    const int64_t ddn = a.ddn;
    const int64_t nch = (ddn + 63) >> 6;
    S *s_row = reinterpret_cast<S *>(smem_raw);
    uint32_t *s_base = reinterpret_cast<uint32_t *>(s_row + (ddn + 1));
    uint32_t *s_w = s_base + nch;
    uint16_t *s_d = reinterpret_cast<uint16_t *>(s_w + nch);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S nt0 = (S)(-a.t0);
    const int T = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t nrow = (uint32_t)ddn;
    for (int64_t j = tid; j < nch; j += T) {
        s_base[j] = a.fb_base[j];
        s_w[j] = a.fb_w[j];
    }
    for (int64_t c = tid; c < ddn; c += T) s_d[c] = (uint16_t)a.dns[c];
    if (tid == 0) s_row[nrow] = (S)0;
    auto load_col = [&](int64_t c, uint4 (&q)[4], uint32_t &nq) {
        nq = 0;
        if (c >= ddn) return;
        const uint32_t wc = s_w[c >> 6];
        nq = wc >> 3;
        const uint4 *p = reinterpret_cast<const uint4 *>(a.fb_ent + s_base[c >> 6] + (uint32_t)(c & 63) * (wc >> 1));
#pragma unroll
        for (int g = 0; g < 4; ++g)
            if ((uint32_t)g < nq) q[g] = p[g];
    };
    const uint32_t rbytes = nrow * NV * (uint32_t)sizeof(S);
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const __amdgpu_buffer_rsrc_t rv = buf_rsrc(v + (size_t)ru * nrow * NV, rbytes);
        const uint32_t uu = a.ups[ru];
        for (int ln = 0; ln < NV; ++ln) {
            for (uint32_t base = 0; base < nrow; base += (uint32_t)E * T) {
                S tv[E];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint32_t i = base + (uint32_t)e * T + tid;
                    tv[e] = buf_ld<S>(rv, ((i < nrow ? i : nrow - 1) * NV + ln) * (uint32_t)sizeof(S));
                }
                if (base == 0) __syncthreads();    // every gather of the previous lane has finished
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint32_t i = base + (uint32_t)e * T + tid;
                    if (i < nrow) s_row[i] = tv[e];
                }
            }
            uint4 cur[4], nxt[4];
            uint32_t ncur, nnxt;
            load_col(tid, cur, ncur);
            __syncthreads();
            for (int64_t c = tid; c < ddn; c += T) {
                load_col(c + T, nxt, nnxt);
                S acc[1] = {(S)0};
                fb_gather<S, 1>(cur, ncur, s_row, acc);
                const S dg = hub_diag<S>(a, uu, (uint32_t)s_d[c]);
                w[((size_t)ru * ddn + c) * NV + ln] = dg * s_row[c] + nt0 * acc[0];
#pragma unroll
                for (int g = 0; g < 4; ++g) cur[g] = nxt[g];
                ncur = nnxt;
            }
        }
    }
}

// Columns kernel of the fast path: the same XCD-queued slab sweep as
// k_hub_cols; staged entries are byte offsets of the neighbour rows. Each
// lane owns CPL adjacent columns (CPL = 2 with one real FP64 vector: one
// 16-byte load per neighbour row, half the requests of CPL = 1; needs an
// even row length). A scalar's summation order does not depend on CPL.
template <typename S, int K>
__device__ __forceinline__ void load_k(const S *p, S (&o)[K])
{
    if constexpr (K * sizeof(S) == 16) {
        const uint4 x = *reinterpret_cast<const uint4 *>(p);
        __builtin_memcpy(o, &x, 16);
    } else if constexpr (K * sizeof(S) == 8) {
        const uint2 x = *reinterpret_cast<const uint2 *>(p);
        __builtin_memcpy(o, &x, 8);
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) o[j] = p[j];
    }
}

// HB (one wave per row, RPW == 1): the row's neighbour count is uniform
// over the wave, so the plus and minus lists are walked as one stream with
// up to kColsBatch loads in flight per round, and the epilogue operands are
// loaded before the first round. Each sum keeps its entry order, so the
// results are bit-identical to the two-list walk. The neighbour rows are
// read with raw buffer loads over V; the slots of a round past the end of
// the list take an offset beyond V's last byte, which the buffer range
// check answers with zeros and no memory request (the sums then add +0,
// which leaves a sum that starts at +0 unchanged).
constexpr int kColsBatch = 12;
// V may take at most this many bytes on the HB path (offset kColsOob is
// out of range, and offset + 16 does not wrap)
constexpr uint32_t kColsOob = 0xFFFFFF00u;

template <typename S, int K>
__device__ __forceinline__ void buf_load_k(__amdgpu_buffer_rsrc_t r, uint32_t off, S (&o)[K])
{
    if constexpr (K * sizeof(S) == 16) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0);
        __builtin_memcpy(o, &x, 16);
    } else if constexpr (K * sizeof(S) == 8) {
        const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0);
        __builtin_memcpy(o, &x, 8);
    } else {
        static_assert(K * sizeof(S) == 4, "one, two or four 32-bit words per lane");
        const auto x = __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0);
        __builtin_memcpy(o, &x, 4);
    }
}

template <typename S, int NV, int CW, bool DOTS, int CPL = 1, bool HB = false>
__global__ __launch_bounds__(256) void k_hub_cols_f(HubKArgs a)
{
    __shared__ double sh_red[4 * 2 * NV + 8];
    __shared__ uint32_t s_ent[kColsLdsEntries];
    __shared__ uint32_t s_off[kColsRows + 1];
    __shared__ uint32_t s_mid[kColsRows];
    __shared__ int s_item;
    __shared__ unsigned s_last;
    const int home = xcc_id();
    const char *__restrict__ vb = static_cast<const char *>(a.v);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *__restrict__ accp = static_cast<S *>(a.acc_out);
    double c1 = 1.0, c2 = 0.0;
    if (a.ecoef) {
        c1 = a.ecoef[0];
        c2 = a.ecoef[1];
    }
    const S c1s = (S)c1, c2s = (S)c2, nt0 = (S)(-a.t0);
    constexpr uint32_t ESZ = NV * sizeof(S);

    const int64_t ddn = a.ddn, dup = a.dup;
    // V as one raw buffer (HB path: the launcher keeps its size below kColsOob)
    const __amdgpu_buffer_rsrc_t rvb = buf_rsrc(a.v, (uint32_t)((uint64_t)dup * (uint64_t)ddn * ESZ));
    const int nchunk = (int)((dup + a.item_rows - 1) / a.item_rows);
    constexpr int LPR = CW / CPL;   // lanes per row
    constexpr int RPW = 64 / LPR;
    constexpr int K = NV * CPL;     // scalars per lane
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int q = home, tries = 0;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) {
            int it = -1;
            while (tries < 8) {
                const int nsl_q = q < a.nslab ? (a.nslab - q + 7) / 8 : 0;
                const int cand = (int)atomicAdd(&a.sched[q], 1u);
                if (cand < nsl_q * nchunk) {
                    it = q + 8 * cand;
                    break;
                }
                q = (q + 1) & 7;
                ++tries;
            }
            s_item = it;
        }
        __syncthreads();
        const int item = s_item;
        if (item < 0) break;
        const int iq = item & 7, idx = item >> 3;
        const int slab = iq + 8 * (idx / nchunk);
        const int chunk = idx % nchunk;
        const int64_t r0 = (int64_t)chunk * a.item_rows;
        const int64_t r1 = r0 + a.item_rows < dup ? r0 + a.item_rows : dup;
        {
            const uint32_t base = a.fu_off[r0];
            for (int64_t i = threadIdx.x; i <= r1 - r0; i += blockDim.x) s_off[i] = a.fu_off[r0 + i] - base;
            for (int64_t i = threadIdx.x; i < r1 - r0; i += blockDim.x) s_mid[i] = a.fu_mid[r0 + i] - base;
            const uint32_t n = a.fu_off[r1] - base;
            for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) s_ent[i] = a.fu_ent[base + i] * ESZ;
        }
        __syncthreads();
        double d0[NV], d1[NV];
#pragma unroll
        for (int j = 0; j < NV; ++j) d0[j] = d1[j] = 0.0;
        const int64_t col = (int64_t)slab * CW + CPL * (lane % LPR);
        const bool colok = col < ddn;
        const uint32_t colb = (uint32_t)col * ESZ;
        for (int64_t r = r0 + wid * RPW + lane / LPR; r < r1; r += 4 * RPW) {
            if (!colok) continue;
            const size_t me = (size_t)(a.row_of ? (int64_t)a.row_of[r] : r) * ddn + col;
            if constexpr (HB) {
                // one wave per row: the list bounds are wave-uniform
                // (scalar); several rows per wave: per lane, and the wave
                // walks until its longest list is done
                uint32_t eb = s_off[r - r0], em = s_mid[r - r0], ee = s_off[r - r0 + 1];
                if constexpr (RPW == 1) {
                    eb = __builtin_amdgcn_readfirstlane(eb);
                    em = __builtin_amdgcn_readfirstlane(em);
                    ee = __builtin_amdgcn_readfirstlane(ee);
                }
                // u is row-uniform (null or not): the same register lanes
                // either way, read from w itself when there is no u
                const S *up = u ? u : w;
                S wv[K], uv[K], vv[K];
#pragma unroll
                for (int j = 0; j < K; ++j) wv[j] = __builtin_nontemporal_load(&w[me * NV + j]);
#pragma unroll
                for (int j = 0; j < K; ++j) uv[j] = __builtin_nontemporal_load(&up[me * NV + j]);
#pragma unroll
                for (int j = 0; j < K; ++j) vv[j] = DOTS ? v[me * NV + j] : (S)0;
                S hp[K], hm[K];
#pragma unroll
                for (int j = 0; j < K; ++j) hp[j] = hm[j] = (S)0;
                // one round: NB loads issued as one group in flight; slots
                // past the list read zeros (out-of-range offset, no
                // request); the sums take each entry once, in order (a lane
                // whose list is done, or empty, reads an entry of the staged
                // lists and discards it)
                const uint32_t elast = ee > 0 ? ee - 1 : 0;
                auto round = [&](auto nb_c, uint32_t e0) {
                    constexpr int NB = decltype(nb_c)::value;
                    uint32_t eo[NB];
#pragma unroll
                    for (int t = 0; t < NB; ++t)
                        eo[t] = e0 + t < ee ? s_ent[e0 + t < ee ? e0 + t : elast] + colb : kColsOob;
                    S nv[NB][K];
#pragma unroll
                    for (int t = 0; t < NB; ++t) buf_load_k<S, K>(rvb, eo[t], nv[t]);
                    // keep the whole group in flight before the first sum
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int t = 0; t < NB; ++t) {
                        const bool plus = e0 + t < em;
#pragma unroll
                        for (int j = 0; j < K; ++j) {
                            hp[j] += plus ? nv[t][j] : (S)0;
                            hm[j] += plus ? (S)0 : nv[t][j];
                        }
                    }
                };
                if constexpr (RPW == 1) {
                    // rounds of kColsBatch, the last one sized to what is
                    // left (8 or 4): fewer issued slots, same order
                    uint32_t e0 = eb;
                    for (; e0 + kColsBatch <= ee; e0 += kColsBatch)
                        round(std::integral_constant<int, kColsBatch>{}, e0);
                    const uint32_t rem = ee - e0;
                    if (rem > 8) round(std::integral_constant<int, kColsBatch>{}, e0);
                    else if (rem > 4) round(std::integral_constant<int, 8>{}, e0);
                    else if (rem > 0) round(std::integral_constant<int, 4>{}, e0);
                } else {
                    for (uint32_t e0 = eb; __ballot(e0 < ee) != 0; e0 += kColsBatch)
                        round(std::integral_constant<int, kColsBatch>{}, e0);
                }
                S hraw[K], hout[K];
#pragma unroll
                for (int j = 0; j < K; ++j) hraw[j] = wv[j] + nt0 * (hp[j] - hm[j]);
                if (a.coef_cplx) {
                    epilogue_r<S, K>(hraw, uv, u != nullptr, 1, a.ecoef, hout);
                } else {
#pragma unroll
                    for (int j = 0; j < K; ++j) hout[j] = c1s * hraw[j];
                    if (u) {
#pragma unroll
                        for (int j = 0; j < K; ++j) hout[j] += c2s * uv[j];
                    }
                }
#pragma unroll
                for (int j = 0; j < K; ++j) __builtin_nontemporal_store(hout[j], &w[me * NV + j]);
                if (accp) {
#pragma unroll
                    for (int j = 0; j < K; ++j)
                        __builtin_nontemporal_store(__builtin_nontemporal_load(&accp[me * NV + j]) + hout[j],
                                                    &accp[me * NV + j]);
                }
                if constexpr (DOTS) {
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const double o = a.dot_raw ? (double)hraw[j] : (double)hout[j];
                        d0[j % NV] += (double)vv[j] * o;
                        d1[j % NV] += o * o;
                    }
                }
                continue;
            }
            S ap[K], am[K];
#pragma unroll
            for (int j = 0; j < K; ++j) ap[j] = am[j] = (S)0;
            const uint32_t eb = s_off[r - r0], em = s_mid[r - r0], ee = s_off[r - r0 + 1];
            uint32_t e = eb;
            for (; e + 8 <= em; e += 8) {
                S nv[8][K];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    load_k<S, K>(reinterpret_cast<const S *>(vb + (s_ent[e + t] + colb)), nv[t]);
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < K; ++j) ap[j] += nv[t][j];
            }
            for (; e < em; ++e) {
                S nv[K];
                load_k<S, K>(reinterpret_cast<const S *>(vb + (s_ent[e] + colb)), nv);
#pragma unroll
                for (int j = 0; j < K; ++j) ap[j] += nv[j];
            }
            for (; e + 8 <= ee; e += 8) {
                S nv[8][K];
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    load_k<S, K>(reinterpret_cast<const S *>(vb + (s_ent[e + t] + colb)), nv[t]);
#pragma unroll
                for (int t = 0; t < 8; ++t)
#pragma unroll
                    for (int j = 0; j < K; ++j) am[j] += nv[t][j];
            }
            for (; e < ee; ++e) {
                S nv[K];
                load_k<S, K>(reinterpret_cast<const S *>(vb + (s_ent[e] + colb)), nv);
#pragma unroll
                for (int j = 0; j < K; ++j) am[j] += nv[j];
            }
            S out[K], raw[K];
#pragma unroll
            for (int j = 0; j < K; ++j) raw[j] = __builtin_nontemporal_load(&w[me * NV + j]) + nt0 * (ap[j] - am[j]);
            if (a.coef_cplx) {
                S uu[K];
                if (u)
#pragma unroll
                    for (int j = 0; j < K; ++j) uu[j] = __builtin_nontemporal_load(&u[me * NV + j]);
                epilogue<S, K>(raw, u ? uu : nullptr, 1, a.ecoef, out);
            } else {
#pragma unroll
                for (int j = 0; j < K; ++j) out[j] = c1s * raw[j];
                if (u) {
#pragma unroll
                    for (int j = 0; j < K; ++j) out[j] += c2s * __builtin_nontemporal_load(&u[me * NV + j]);
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j) __builtin_nontemporal_store(out[j], &w[me * NV + j]);
            if (accp) {
#pragma unroll
                for (int j = 0; j < K; ++j)
                    __builtin_nontemporal_store(__builtin_nontemporal_load(&accp[me * NV + j]) + out[j],
                                                &accp[me * NV + j]);
            }
            if constexpr (DOTS) {
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const double o = a.dot_raw ? (double)raw[j] : (double)out[j];
                    d0[j % NV] += (double)v[me * NV + j] * o;
                    d1[j % NV] += o * o;
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
            if (threadIdx.x == 0) {
                const size_t slot = (size_t)slab * nchunk + chunk;
                for (int j = 0; j < 2 * NV; ++j) a.red.partial[slot * 2 * NV + j] = vals[j];
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        s_last = (atomicAdd(&a.sched[8], 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    if constexpr (DOTS) {
        const size_t nitems = (size_t)a.nslab * nchunk;
        for (int j = 0; j < 2 * NV; ++j) {
            double s = 0.0;
            for (size_t it = threadIdx.x; it < nitems; it += blockDim.x)
                s += __builtin_nontemporal_load(&a.red.partial[it * 2 * NV + j]);
            double vv[1] = {s};
            block_sum<1>(vv, sh_red);
            if (threadIdx.x == 0) a.red.result[j] = vv[0];
        }
    }
    if (threadIdx.x == 0) {
        for (int i = 0; i < 8; ++i) a.sched[i] = 0u;
        a.sched[8] = 0u;
        __threadfence();
    }
}


// ------------------------------------------------------------ tile T_up --
// T_up with the rows of one up block staged in LDS (uniform |t|, one real
// vector, even row length). The up rows split by the top `tile bits` sites
// of the up configuration into blocks of consecutive rows; a hop that
// leaves those sites alone keeps its target in the block ("local"), the
// others change the block ("far"). A work item is (slab of kTileCols
// columns, block): the block's rows of the slab are staged once (eight lanes
// per row segment, two columns each), the local hops read LDS and only the
// far hops gather from L2/HBM. Items are taken slab-major from per-XCD
// queues, so all blocks of a slab -- the rows the far hops read -- pass
// through one XCD's L2 close together. Each thread reads its row's lists
// itself (16-byte groups of four entries, L2-resident: every slab of a
// block reuses them), so the passes over the block need no barrier; the
// LDS holds the staged rows only, and small blocks let several workgroups
// share a CU. Rows are processed in an order that groups equal hop counts
// (less divergence among the eight rows of a wave); each element's sum
// keeps the table's entry order, and the fused dots are per-item partials
// summed in item order by the last workgroup.
constexpr int kTileCols = 16;        // columns per slab (8 lanes x 2)
constexpr int kTileSlots = 128;      // rows per pass (1024 threads / 8 lanes)
constexpr int kTileLocalGroups = 3;  // 8-entry groups of local hops per row (16-bit)
constexpr int kTileFar = 12;         // far hops per row
// LDS behind the staged rows: block reduction scratch (16 waves x 2), item
// and last-group words
constexpr uint32_t kTileTailBytes = 8u * 32 + 16;
template <typename S> constexpr int tile_row_stride() { return kTileCols + 16 / (int)sizeof(S); }

template <typename S> struct Pair;
template <> struct Pair<double> { using T = double2; };
template <> struct Pair<float> { using T = float2; };
// two adjacent elements through the nontemporal path (streams touched once)
template <typename S> __device__ __forceinline__ typename Pair<S>::T nt_load2(const S *p)
{
    typedef S v2 __attribute__((ext_vector_type(2)));
    const v2 x = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    typename Pair<S>::T o;
    o.x = x.x;
    o.y = x.y;
    return o;
}
template <typename S> __device__ __forceinline__ void nt_store2(S *p, S a, S b)
{
    typedef S v2 __attribute__((ext_vector_type(2)));
    v2 x;
    x.x = a;
    x.y = b;
    __builtin_nontemporal_store(x, reinterpret_cast<v2 *>(p));
}

template <typename S, bool DOTS>
__global__ __launch_bounds__(1024) void k_hub_up_tile(HubKArgs a)
{
    extern __shared__ unsigned char smem_raw[];
    using P2 = typename Pair<S>::T;
    constexpr int RS = tile_row_stride<S>();
    S *tile = reinterpret_cast<S *>(smem_raw);
    double *sh_red = reinterpret_cast<double *>(smem_raw + a.ft_tile_bytes);
    int *s_item = reinterpret_cast<int *>(sh_red + 32);
    unsigned *s_last = reinterpret_cast<unsigned *>(s_item + 1);
    const int home = xcc_id();
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    const uint4 *__restrict__ ent4 = reinterpret_cast<const uint4 *>(a.ft_ent);
    double c1 = 1.0, c2 = 0.0;
    if (a.ecoef) {
        c1 = a.ecoef[0];
        c2 = a.ecoef[1];
    }
    const S c1s = (S)c1, c2s = (S)c2, nt0 = (S)(-a.t0);
    const int64_t ddn = a.ddn, ld = a.ld;
    const int tid = threadIdx.x, l8 = tid & 7, slot = tid >> 3;
    const int nb = a.ft_nb;
    int q = home, tries = 0;
    for (;;) {
        __syncthreads();    // the previous item's readers of the staged rows are done
        if (tid == 0) {
            int it = -1;
            while (tries < 8) {
                const int nsl_q = q < a.nslab ? (a.nslab - q + 7) / 8 : 0;
                const int cand = (int)atomicAdd(&a.sched[q], 1u);
                if (cand < nsl_q * nb) {
                    it = q + 8 * cand;
                    break;
                }
                q = (q + 1) & 7;
                ++tries;
            }
            *s_item = it;
        }
        __syncthreads();
        const int item = *s_item;
        if (item < 0) break;
        const int idx = item >> 3;
        const int slab = (item & 7) + 8 * (idx / nb);
        const int blk = idx % nb;
        const int64_t r0 = a.ft_blk[blk], nr = (int64_t)a.ft_blk[blk + 1] - r0;
        const int64_t col = (int64_t)slab * kTileCols + 2 * l8;
        const bool cok = col < ddn;    // an even row length: both columns or neither
        // stage the block's rows of the slab: four row loads per thread in
        // flight, then their LDS stores (a load-store pair per row waits out
        // one memory round trip per row; eight in flight spill registers)
        for (int64_t i0 = slot; i0 < nr; i0 += 4 * kTileSlots) {
            P2 x[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = i0 + (int64_t)t * kTileSlots;
                x[t].x = (S)0;
                x[t].y = (S)0;
                if (cok && i < nr) x[t] = *reinterpret_cast<const P2 *>(v + (size_t)(r0 + i) * ld + col);
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int64_t i = i0 + (int64_t)t * kTileSlots;
                if (i < nr) *reinterpret_cast<P2 *>(tile + i * RS + 2 * l8) = x[t];
            }
        }
        __syncthreads();
        double dv = 0.0, dd = 0.0;
        // software pipeline over this thread's rows of the block: a row's
        // position data are loaded two passes ahead and its far entries one
        // pass ahead; a pass issues its far gathers, epilogue operands and
        // local entry groups together, then reads the local hops from LDS
        uint32_t lr_n = 0, cnt_n = 0, off_n = 0;
        if (slot < nr) {
            lr_n = a.ft_pos[r0 + slot];
            cnt_n = a.ft_cnt[r0 + slot];
            off_n = a.ft_off[r0 + slot];
        }
        // a row's far entries are loaded one pass ahead (its position data
        // two passes ahead), so a pass issues its far gathers at once
        uint32_t lr_nn = 0, cnt_nn = 0, off_nn = 0;
        uint4 fe_n[kTileFar / 4];
        auto load_far = [&](uint32_t c, uint32_t o, uint4 *dst) {
            const uint32_t nlc = (c & 255u) + ((c >> 8) & 255u), nfc = ((c >> 16) & 255u) + (c >> 24);
            const uint32_t glc = (nlc + 7) >> 3, gfc = (nfc + 3) >> 2;
#pragma unroll
            for (int g = 0; g < kTileFar / 4; ++g) {
                dst[g] = make_uint4(0u, 0u, 0u, 0u);
                if ((uint32_t)g < gfc) dst[g] = ent4[(o >> 2) + glc + g];
            }
        };
        if (slot < nr && cok) load_far(cnt_n, off_n, fe_n);
        if (slot + kTileSlots < nr) {
            lr_nn = a.ft_pos[r0 + slot + kTileSlots];
            cnt_nn = a.ft_cnt[r0 + slot + kTileSlots];
            off_nn = a.ft_off[r0 + slot + kTileSlots];
        }
        for (int64_t p = slot; p < nr && cok; p += kTileSlots) {
            const uint32_t lr = lr_n, cnt = cnt_n, g0 = off_n >> 2;
            uint4 fe[kTileFar / 4];
#pragma unroll
            for (int g = 0; g < kTileFar / 4; ++g) fe[g] = fe_n[g];
            lr_n = lr_nn;
            cnt_n = cnt_nn;
            off_n = off_nn;
            if (p + kTileSlots < nr) load_far(cnt_n, off_n, fe_n);
            if (p + 2 * kTileSlots < nr) {
                lr_nn = a.ft_pos[r0 + p + 2 * kTileSlots];
                cnt_nn = a.ft_cnt[r0 + p + 2 * kTileSlots];
                off_nn = a.ft_off[r0 + p + 2 * kTileSlots];
            }
            // the epilogue streams (w in and out, u) are touched once: kept
            // out of the way of the slab's rows in L2
            const size_t me = (size_t)(r0 + lr) * ld + col;
            const P2 wv = nt_load2<S>(w + me);
            P2 uv;
            uv.x = (S)0;
            uv.y = (S)0;
            if (u) uv = nt_load2<S>(u + me);
            // entries in 16-byte groups: local (plus then minus), then far
            // (plus then minus) from the next group boundary; at most
            // kTileLocalGroups local groups and kTileFar far entries per
            // row (checked when the tables are built)
            const uint32_t nlp = cnt & 255u, nl = nlp + ((cnt >> 8) & 255u);
            const uint32_t nfp = (cnt >> 16) & 255u, nf = nfp + (cnt >> 24);
            // local entries are 16-bit (eight per group), far ones 32-bit
            const uint32_t ngl = (nl + 7) >> 3;
            uint4 le[kTileLocalGroups];
#pragma unroll
            for (int g = 0; g < kTileLocalGroups; ++g) {
                le[g] = make_uint4(0u, 0u, 0u, 0u);
                if ((uint32_t)g < ngl) le[g] = ent4[g0 + g];
            }
            S p0v = (S)0, p1v = (S)0, m0v = (S)0, m1v = (S)0;
            // far gathers in batches of eight, the first batch in flight
            // while the local reads run
            auto far_batch = [&](auto b0_c, P2 (&fx)[8]) {
                constexpr int b0 = decltype(b0_c)::value;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (b0 + t >= kTileFar) break;
                    const uint4 g4 = fe[(b0 + t) >> 2];
                    const uint32_t e = ((b0 + t) & 3) == 0 ? g4.x : ((b0 + t) & 3) == 1 ? g4.y
                                     : ((b0 + t) & 3) == 2 ? g4.z : g4.w;
                    fx[t].x = (S)0;
                    fx[t].y = (S)0;
                    if ((uint32_t)(b0 + t) < nf) fx[t] = *reinterpret_cast<const P2 *>(v + (size_t)e * ld + col);
                }
            };
            auto far_sum = [&](auto b0_c, const P2 (&fx)[8]) {
                constexpr int b0 = decltype(b0_c)::value;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    if (b0 + t >= kTileFar) break;
                    if ((uint32_t)(b0 + t) < nfp) {
                        p0v += fx[t].x;
                        p1v += fx[t].y;
                    } else if ((uint32_t)(b0 + t) < nf) {
                        m0v += fx[t].x;
                        m1v += fx[t].y;
                    }
                }
            };
            P2 fx[8];
            far_batch(std::integral_constant<int, 0>{}, fx);
#pragma unroll
            for (int g = 0; g < kTileLocalGroups; ++g) {
                const uint32_t e4[4] = {le[g].x, le[g].y, le[g].z, le[g].w};
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const uint32_t k = 8u * g + t;
                    if (k < nl) {
                        // one 16-byte read: a row group's eight lanes read
                        // one contiguous 128-byte row segment per pass
                        const P2 tv = *reinterpret_cast<const P2 *>(
                            tile + ((e4[t >> 1] >> (16 * (t & 1))) & 0xFFFFu) * RS + 2 * l8);
                        if (k < nlp) {
                            p0v += tv.x;
                            p1v += tv.y;
                        } else {
                            m0v += tv.x;
                            m1v += tv.y;
                        }
                    }
                }
            }
            far_sum(std::integral_constant<int, 0>{}, fx);
            if (nf > 8) {
                far_batch(std::integral_constant<int, 8>{}, fx);
                far_sum(std::integral_constant<int, 8>{}, fx);
            }
            const S raw0 = wv.x + nt0 * (p0v - m0v), raw1 = wv.y + nt0 * (p1v - m1v);
            S o0 = c1s * raw0 + c2s * uv.x, o1 = c1s * raw1 + c2s * uv.y;
            if (!u) {
                o0 = c1s * raw0;
                o1 = c1s * raw1;
            }
            nt_store2<S>(w + me, o0, o1);
            if constexpr (DOTS) {
                const S *tp = tile + lr * RS + 2 * l8;
                const double x0 = a.dot_raw ? (double)raw0 : (double)o0;
                const double x1 = a.dot_raw ? (double)raw1 : (double)o1;
                dv += (double)tp[0] * x0 + (double)tp[1] * x1;
                dd += x0 * x0 + x1 * x1;
            }
        }
        if constexpr (DOTS) {
            double vals[2] = {dv, dd};
            block_sum<2>(vals, sh_red);
            if (tid == 0) {
                const size_t sl = (size_t)slab * nb + blk;
                a.red.partial[2 * sl] = vals[0];
                a.red.partial[2 * sl + 1] = vals[1];
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        *s_last = (atomicAdd(&a.sched[8], 1u) == gridDim.x - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
    if constexpr (DOTS) {
        const size_t nitems = (size_t)a.nslab * nb;
        for (int j = 0; j < 2; ++j) {
            double sum = 0.0;
            for (size_t it = tid; it < nitems; it += blockDim.x)
                sum += __builtin_nontemporal_load(&a.red.partial[it * 2 + j]);
            double vv[1] = {sum};
            block_sum<1>(vv, sh_red);
            if (tid == 0) a.red.result[j] = vv[0];
        }
    }
    if (tid == 0) {
        for (int i = 0; i < 8; ++i) a.sched[i] = 0u;
        a.sched[8] = 0u;
        __threadfence();
    }
}

template <typename S, int NV, int CW>
static void launch_cols_t(const HubKArgs &a, int grid, hipStream_t st)
{
    if constexpr (NV == 2) {
        if (a.coef_im) {
            if (a.nd) hipLaunchKernelGGL((k_hub_cols<S, 2, CW, true, true>), dim3(grid), dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_hub_cols<S, 2, CW, false, true>), dim3(grid), dim3(256), 0, st, a);
            return;
        }
    }
    if (a.nd) hipLaunchKernelGGL((k_hub_cols<S, NV, CW, true>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_hub_cols<S, NV, CW, false>), dim3(grid), dim3(256), 0, st, a);
}

template <typename S, int NV, int CW>
static void launch_cols_f(const HubKArgs &a, int grid, hipStream_t st)
{
    if (a.row_cols == 2 && NV == 1) {
        if constexpr (CW >= 16 && NV == 1) {
            if (a.hb) {
                // batched walk, 64 / (CW / 2) rows per wave
                if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, true, 2, true>), dim3(grid), dim3(256), 0, st, a);
                else hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, false, 2, true>), dim3(grid), dim3(256), 0, st, a);
                return;
            }
        }
        if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, true, 2>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, false, 2>), dim3(grid), dim3(256), 0, st, a);
        return;
    }
    if constexpr (CW == 64) {
        if (a.hb) {
            if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, NV, 64, true, 1, true>), dim3(grid), dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_hub_cols_f<S, NV, 64, false, 1, true>), dim3(grid), dim3(256), 0, st, a);
            return;
        }
    }
    if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, true>), dim3(grid), dim3(256), 0, st, a);
    else hipLaunchKernelGGL((k_hub_cols_f<S, NV, CW, false>), dim3(grid), dim3(256), 0, st, a);
}

template <typename S, int NV>
static void launch_cols_f128(const HubKArgs &a, int grid, hipStream_t st)
{
    if constexpr (NV == 1) {
        if (a.hb) {
            if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, 1, 128, true, 2, true>), dim3(grid), dim3(256), 0, st, a);
            else hipLaunchKernelGGL((k_hub_cols_f<S, 1, 128, false, 2, true>), dim3(grid), dim3(256), 0, st, a);
            return;
        }
        if (a.nd) hipLaunchKernelGGL((k_hub_cols_f<S, 1, 128, true, 2>), dim3(grid), dim3(256), 0, st, a);
        else hipLaunchKernelGGL((k_hub_cols_f<S, 1, 128, false, 2>), dim3(grid), dim3(256), 0, st, a);
    }
}

// The rows kernel with the fused Lanczos update runs where the batched
// hop-ordered rows kernel runs (hub_row_cols 5 or 6) on one real vector
// with at most 13 row elements per lane.
static size_t rows_fz_bytes(int64_t ddn, size_t esz)
{
    return (size_t)(ddn + 1) * esz + 8 * (size_t)((ddn + 63) / 64) + 2 * (size_t)ddn + kRowsFzTail;
}
bool hub_rows_fused_ok(hphi_ham *h, int nv)
{
    if (h->kind != 1 || nv != 1 || !h->hub.uniform_t || !h->hub.fb_ok) return false;
    const int rc = h->sched_cfg.hub_row_cols;
    if ((rc != 5 && rc != 6) || h->basis->n_sites > 16) return false;
    const int64_t dup = h->basis->sp[0].dim, ddn = h->basis->sp[1].dim;
    if (ddn > 13 * 1024) return false;    // row elements per lane of k_hub_rows_fz
    if (rows_fz_bytes(ddn, sizeof(double)) > 160 * 1024) return false;
    return (unsigned __int128)dup * ddn * sizeof(double) < ((unsigned __int128)1 << 32);
}

// True when every kernel that reads pre-scaled slot words has no static
// LDS, so that its dynamic LDS (the row) starts at LDS address 0.
template <typename S>
static bool fc_kernels_lds0()
{
    static const bool ok = [] {
        const void *ks[] = {(const void *)k_hub_rows_fp<S, 1, 16, true>, (const void *)k_hub_rows_fz<S, 8, true>,
                            (const void *)k_hub_rows_fz<S, 13, true>};
        for (const void *k : ks) {
            hipFuncAttributes fa{};
            if (hipFuncGetAttributes(&fa, k) != hipSuccess || fa.sharedSizeBytes != 0) return false;
        }
        return true;
    }();
    return ok;
}

template <typename S, int NV>
static int launch_hub_t(hphi_ham *h, HubKArgs a, hipStream_t st)
{
    const int ncu = h->basis->ctx->n_cu > 0 ? h->basis->ctx->n_cu : 256;
    // rows kernel
    const bool cx = NV == 2 && a.coef_im;   // complex class values
    size_t row_bytes = (size_t)a.ddn * NV * sizeof(S) + (cx ? 256 : 128) * sizeof(S);
    bool lds_row = row_bytes <= 160 * 1024;
    int per_cu = lds_row ? (int)((160 * 1024) / row_bytes) : 4;
    if (per_cu < 1) per_cu = 1;
    if (per_cu > 4) per_cu = 4;
    int64_t grid_r = (int64_t)ncu * per_cu;
    if (grid_r > a.dup) grid_r = a.dup;
    int threads = 1024;
    const size_t fast_row_bytes = (size_t)(a.ddn + 1) * NV * sizeof(S);
    // uniform |t| tables and 32-bit byte offsets: the fast column kernels;
    // the fast rows kernels also need the whole NV-lane row in LDS
    const bool fast_cols = h->hub.uniform_t &&
                           (unsigned __int128)a.dup * a.ddn * NV * sizeof(S) < ((unsigned __int128)1 << 32);
    const bool fast = fast_cols && fast_row_bytes <= 160 * 1024;
    const int rmode = h->sched_cfg.hub_row_cols;
    const size_t fm_bytes = fast_row_bytes + 8 * (size_t)((a.ddn + 63) / 64) + 2 * (size_t)a.ddn + 16;
    // one lane of the row in LDS (rows kernel for wide rows of NV > 1 lanes)
    const size_t fl_bytes = (size_t)(a.ddn + 1) * sizeof(S) + 8 * (size_t)((a.ddn + 63) / 64) + 2 * (size_t)a.ddn + 16;
    const bool lane_rows = NV > 1 && !fast && fast_cols && rmode >= 4 && h->hub.fb_ok && fl_bytes <= 160 * 1024 &&
                           h->basis->n_sites <= 16;
    // hub_row_cols 6: the batched hop-ordered rows kernels read pre-scaled
    // slot words (one real vector; otherwise as 5). Their LDS addresses
    // assume the row at LDS address 0: no static LDS in those kernels.
    const bool fc_rows = rmode == 6 && NV == 1 && h->hub.fc_ok && fc_kernels_lds0<S>();
    a.fc_ent = fc_rows ? h->hub.fc_ent[sizeof(S) == 8 ? 1 : 0].as<uint32_t>() : nullptr;
    const bool rows_fp_fc = fc_rows && fast && fm_bytes <= 160 * 1024 && h->basis->n_sites <= 16 &&
                            a.ddn <= 16 * (int64_t)threads;
    const bool rows_fp = fast && rmode >= 5 && h->hub.fb_ok && fm_bytes <= 160 * 1024 && h->basis->n_sites <= 16 &&
                         a.ddn * NV <= 16 * (int64_t)threads;
    // the T_up tile kernel (hub_sweep 7)
    const size_t tile_bytes = (size_t)h->hub.ft_max_rows * tile_row_stride<S>() * sizeof(S);
    const bool tile = h->sched_cfg.hub_sweep == 7 && NV == 1 && fast_cols && !a.coef_cplx && !a.acc_out &&
                      h->hub.ft_ok && a.ddn % 2 == 0 && a.ld % 2 == 0 && tile_bytes + kTileTailBytes <= 160 * 1024;
    if (a.ld != a.ddn && !(NV == 1 && tile && (a.lz_q || rows_fp_fc || rows_fp)))
        return fail(HPHI_ERR_UNSUPPORTED, "padded rows need the tile T_up kernel and the batched rows kernels");
    if (a.lz_q) {
        // fused Lanczos update: only where hub_rows_fused_ok holds
        if constexpr (NV == 1) {
            if (!hub_rows_fused_ok(h, 1))
                return fail(HPHI_ERR_UNSUPPORTED, "fused Lanczos update outside its kernel range");
            const size_t fz_bytes = rows_fz_bytes(a.ddn, sizeof(S));
            auto go = [&](auto kern) {
                hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fz_bytes);
                hipLaunchKernelGGL(kern, dim3((unsigned)grid_r), dim3(threads), fz_bytes, st, a);
            };
            const int64_t per = (a.ddn + threads - 1) / threads;
            if (fc_rows) {
                if (per <= 8) go(k_hub_rows_fz<S, 8, true>);
                else go(k_hub_rows_fz<S, 13, true>);
            } else {
                if (per <= 8) go(k_hub_rows_fz<S, 8>);
                else go(k_hub_rows_fz<S, 13>);
            }
        } else {
            return fail(HPHI_ERR_UNSUPPORTED, "fused Lanczos update takes one real vector");
        }
    } else if (lane_rows) {
        if constexpr (NV > 1) {
            hipFuncSetAttribute((const void *)k_hub_rows_fl<S, NV, 13>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)fl_bytes);
            hipLaunchKernelGGL((k_hub_rows_fl<S, NV, 13>), dim3((unsigned)std::min<int64_t>(ncu, a.dup)),
                               dim3(threads), fl_bytes, st, a);
        }
    } else if (rows_fp_fc) {
        hipFuncSetAttribute((const void *)k_hub_rows_fp<S, 1, 16, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fm_bytes);
        hipLaunchKernelGGL((k_hub_rows_fp<S, 1, 16, true>), dim3((unsigned)grid_r), dim3(threads), fm_bytes, st, a);
    } else if (rows_fp) {
        hipFuncSetAttribute((const void *)k_hub_rows_fp<S, NV, 16>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fm_bytes);
        hipLaunchKernelGGL((k_hub_rows_fp<S, NV, 16>), dim3((unsigned)grid_r), dim3(threads), fm_bytes, st, a);
    } else if (fast && rmode >= 4 && h->hub.fb_ok && fm_bytes <= 160 * 1024 && h->basis->n_sites <= 16) {
        hipFuncSetAttribute((const void *)k_hub_rows_fb<S, NV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fm_bytes);
        hipLaunchKernelGGL((k_hub_rows_fb<S, NV>), dim3((unsigned)grid_r), dim3(threads), fm_bytes, st, a);
    } else if (fast && rmode >= 3 && fm_bytes <= 160 * 1024 && h->basis->n_sites <= 16) {
        hipFuncSetAttribute((const void *)k_hub_rows_fm<S, NV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fm_bytes);
        hipLaunchKernelGGL((k_hub_rows_fm<S, NV>), dim3((unsigned)grid_r), dim3(threads), fm_bytes, st, a);
    } else if (fast) {
        hipFuncSetAttribute((const void *)k_hub_rows_f<S, NV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)fast_row_bytes);
        hipLaunchKernelGGL((k_hub_rows_f<S, NV>), dim3((unsigned)grid_r), dim3(threads), fast_row_bytes, st, a);
    } else if (cx) {
        if constexpr (NV == 2) {
            const size_t cl_bytes = (size_t)(a.ddn + 256) * sizeof(S);
            if (!lds_row && cl_bytes <= 160 * 1024) {
                hipFuncSetAttribute((const void *)k_hub_rows_cl<S>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)cl_bytes);
                hipLaunchKernelGGL((k_hub_rows_cl<S>), dim3((unsigned)std::min<int64_t>(ncu, a.dup)),
                                   dim3(threads), cl_bytes, st, a);
            } else if (lds_row) {
                hipFuncSetAttribute((const void *)k_hub_rows<S, 2, true, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)row_bytes);
                hipLaunchKernelGGL((k_hub_rows<S, 2, true, true>), dim3((unsigned)grid_r), dim3(threads),
                                   row_bytes, st, a);
            } else {
                hipLaunchKernelGGL((k_hub_rows<S, 2, false, true>), dim3((unsigned)grid_r), dim3(threads),
                                   256 * sizeof(S), st, a);
            }
        }
    } else if (lds_row) {
        hipFuncSetAttribute((const void *)k_hub_rows<S, NV, true>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)row_bytes);
        hipLaunchKernelGGL((k_hub_rows<S, NV, true>), dim3((unsigned)grid_r), dim3(threads),
                           row_bytes, st, a);
    } else {
        hipLaunchKernelGGL((k_hub_rows<S, NV, false>), dim3((unsigned)grid_r), dim3(threads),
                           128 * sizeof(S), st, a);
    }
    HPHI_HIP(hipGetLastError());
    // two-body terms (exchange, pair hopping, inter-site Coulomb, Hund) add
    // into the partial product before the T_up kernel completes it
    HPHI_TRY(launch_hub_pairs(h, (int)sizeof(S), NV, a.v, a.w, a.ld, st));
    if (a.ev_mid) HPHI_HIP(hipEventRecord(a.ev_mid, st));
    // column kernel, geometry from the Hamiltonian's schedule
    const int cw = h->sched_cfg.hub_slab_cols;
    const int groups = h->sched_cfg.hub_groups;
    if (tile) {
        if constexpr (NV == 1) {
            a.ft_blk = h->hub.ft_blk.as<uint32_t>();
            a.ft_pos = h->hub.ft_pos.as<uint32_t>();
            a.ft_off = h->hub.ft_off.as<uint32_t>();
            a.ft_cnt = h->hub.ft_cnt.as<uint32_t>();
            a.ft_ent = h->hub.ft_ent.as<uint32_t>();
            a.ft_nb = h->hub.ft_nb;
            a.ft_tile_bytes = (uint32_t)((tile_bytes + 15) & ~(size_t)15);
            a.nslab = (int)((a.ddn + kTileCols - 1) / kTileCols);
            const int64_t nitems = (int64_t)a.nslab * a.ft_nb;
            if (a.nd && nitems * 2 > (int64_t)kReduceSlots)
                return fail(HPHI_ERR_UNSUPPORTED, "Hubbard tile items beyond the reduction scratch");
            a.sched = h->sched.as<unsigned>();
            const size_t lds = a.ft_tile_bytes + kTileTailBytes;
            // as many 1024-thread workgroups per CU as the LDS holds (at
            // most two: registers), spread over every XCD
            const int per_cu = std::max(1, std::min(2, (int)((160 * 1024) / lds)));
            const int grid_t = 8 * std::max(1, std::min(groups, per_cu * ncu / 8));
            auto go = [&](auto kern) {
                hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
                hipLaunchKernelGGL(kern, dim3(grid_t), dim3(1024), lds, st, a);
            };
            if (a.nd) go(k_hub_up_tile<S, true>);
            else go(k_hub_up_tile<S, false>);
            HPHI_HIP(hipGetLastError());
            return HPHI_OK;
        }
    }
    if (fast_cols && h->sched_cfg.hub_row_order == 2 && h->hub.rr_row.p) {
        // reverse Cuthill-McKee processing order: lists by position, row map
        a.fu_off = h->hub.rr_off.as<uint32_t>();
        a.fu_mid = h->hub.rr_mid.as<uint32_t>();
        a.fu_ent = h->hub.rr_ent.as<uint32_t>();
        a.row_of = h->hub.rr_row.as<uint32_t>();
    }
    int item_rows = h->sched_cfg.hub_item_rows;
    // the item's neighbour lists must fit the staging array
    while (item_rows > 8 && (int64_t)item_rows * h->hub.max_deg[0] > kColsLdsEntries) item_rows /= 2;
    if ((int64_t)item_rows * h->hub.max_deg[0] > kColsLdsEntries)
        return fail(HPHI_ERR_UNSUPPORTED, "Hubbard up-species degree %lld too large for staging",
                    (long long)h->hub.max_deg[0]);
    a.item_rows = item_rows;
    a.groups = groups;
    // hub_sweep 3 and 5: two adjacent columns per lane (even row length
    // only); 5 also walks each row's lists in batches (one wave per row)
    // hub_sweep 7 where the tile kernel does not apply runs as 5
    const int sw = h->sched_cfg.hub_sweep == 7 ? 5 : h->sched_cfg.hub_sweep;
    a.row_cols = ((sw == 3 || sw == 5) && NV == 1 && a.ddn % 2 == 0) ? 2 : 1;
    a.hb = (sw == 5 && (uint64_t)a.dup * (uint64_t)a.ddn * NV * sizeof(S) <= kColsOob) ? 1 : 0;
    // 128-column slabs only with two columns per lane (one wave per row)
    const int cw_eff = (cw == 128 && !(fast_cols && a.row_cols == 2)) ? 64 : cw;
    a.nslab = (int)((a.ddn + cw_eff - 1) / cw_eff);
    const int64_t grid_c = 8 * (int64_t)groups;
    const int64_t nitems = (int64_t)a.nslab * ((a.dup + item_rows - 1) / item_rows);
    if (a.nd && nitems * 2 * NV > (int64_t)kReduceSlots)
        return fail(HPHI_ERR_UNSUPPORTED, "Hubbard column items beyond the reduction scratch");
    a.sched = h->sched.as<unsigned>();
    if (fast_cols) {
        switch (cw_eff) {
        case 8: launch_cols_f<S, NV, 8>(a, (int)grid_c, st); break;
        case 128: launch_cols_f128<S, NV>(a, (int)grid_c, st); break;
        case 16: launch_cols_f<S, NV, 16>(a, (int)grid_c, st); break;
        case 32: launch_cols_f<S, NV, 32>(a, (int)grid_c, st); break;
        default: launch_cols_f<S, NV, 64>(a, (int)grid_c, st); break;
        }
        HPHI_HIP(hipGetLastError());
        return HPHI_OK;
    }
    switch (cw_eff) {
    case 8: launch_cols_t<S, NV, 8>(a, (int)grid_c, st); break;
    case 16: launch_cols_t<S, NV, 16>(a, (int)grid_c, st); break;
    case 32: launch_cols_t<S, NV, 32>(a, (int)grid_c, st); break;
    default: launch_cols_t<S, NV, 64>(a, (int)grid_c, st); break;
    }
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int64_t hub_lanczos_pitch(hphi_ham *h, int dtype)
{
    const int64_t ddn = h->basis->sp[1].dim, dup = h->basis->sp[0].dim;
    if (h->kind != 1 || h->sched_cfg.hub_sweep != 7 || !h->hub.ft_ok || ddn % 2) return ddn;
    if ((dtype != HPHI_F64 && dtype != HPHI_F32) || !hub_rows_fused_ok(h, 1)) return ddn;
    const size_t esz = dtype_is_f32(dtype) ? 4 : 8;
    const int64_t line = (int64_t)(128 / esz);
    const int64_t ld = (ddn + line - 1) / line * line;
    // the rows kernels' raw buffer offsets stay 32-bit
    if ((unsigned __int128)dup * ld * esz >= ((unsigned __int128)1 << 32)) return ddn;
    const size_t tile_bytes = (size_t)h->hub.ft_max_rows * (esz == 8 ? tile_row_stride<double>() * 8 : tile_row_stride<float>() * 4);
    if (tile_bytes + kTileTailBytes > 160 * 1024) return ddn;
    // the first product's rows kernel must take the pitch too
    const size_t fm_bytes = (size_t)(ddn + 1) * esz + 8 * (size_t)((ddn + 63) / 64) + 2 * (size_t)ddn + 16;
    if (fm_bytes > 160 * 1024 || ddn > 16 * 1024) return ddn;
    return ld;
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
    a.fs_base = h->hub.fs_base.as<uint32_t>();
    a.fs_wp = h->hub.fs_wp.as<uint32_t>();
    a.fs_wm = h->hub.fs_wm.as<uint32_t>();
    a.fs_ent = h->hub.fs_ent.as<uint16_t>();
    a.fu_off = h->hub.fu_off.as<uint32_t>();
    a.fu_mid = h->hub.fu_mid.as<uint32_t>();
    a.fu_ent = h->hub.fu_ent.as<uint32_t>();
    a.fb_base = h->hub.fb_base.as<uint32_t>();
    a.fb_w = h->hub.fb_w.as<uint32_t>();
    a.fb_ent = h->hub.fb_ent.as<uint32_t>();
    a.t0 = h->hub.t0;
    a.coef_im = h->hub.cplx ? h->hub.coef_im.as<double>() : nullptr;
    a.coef_cplx = m.coef_cplx;
    a.lz = m.lz;
    a.lz_alpha = m.lz_alpha;
    a.lz_beta = m.lz_beta;
    a.lz_q = m.lz_q;
    a.lz_red = m.lz_red;
    a.ev_mid = m.ev_mid;
    a.ld = m.ld > 0 ? m.ld : a.ddn;
    if (a.ld < a.ddn) return fail(HPHI_ERR_INVALID_ARG, "row pitch %lld below the row length", (long long)a.ld);
    const int nv = m.nvec * dtype_lanes(m.dtype);
    const bool f32 = dtype_is_f32(m.dtype);
    if (h->hub.cplx && dtype_lanes(m.dtype) != 2)
        return fail(HPHI_ERR_UNSUPPORTED, "complex transfer amplitudes act on complex vectors only");
    if (nv == 1) return f32 ? launch_hub_t<float, 1>(h, a, m.stream) : launch_hub_t<double, 1>(h, a, m.stream);
    if (nv == 2) return f32 ? launch_hub_t<float, 2>(h, a, m.stream) : launch_hub_t<double, 2>(h, a, m.stream);
    return fail(HPHI_ERR_UNSUPPORTED, "Hubbard H*v supports one real or one complex vector per call");
}

} // namespace hphi

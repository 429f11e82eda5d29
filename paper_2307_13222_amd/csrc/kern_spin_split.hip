// Spin H*v split by bond locality (HPhi update paper Sec. 3.2 Heisenberg
// model; cTPQ blocks of Sec. 3.5.1 are its main user).
//
// A sector state x = (h, l) (high and low halves of the sites) sits at
// hi_off[h] + lo_rank[l]: the states of one high pattern h form a block in
// which l runs in lo_rank order, and all blocks whose h has the same
// popcount (a class) have the same length and the same l order. So a bond
// with both ends in the high half maps (h, l) to (h ^ m, l): the same
// position p = lo_rank[l] in another block of the same class. The product
// runs in two passes:
//   A  the stored-list kernel with the other bonds only (both ends low:
//      gathers inside the state's own block; crossing bonds) and the
//      fields, writing the partial product;
//   B  this kernel: the high bonds, in slab order. A wave takes one block
//      h and P consecutive positions p (LPS lanes per state, 16 bytes
//      each); the block's active high bonds and its high-bond diagonal are
//      wave-uniform, and every gather V[hi_off[h ^ m] + p] is one
//      contiguous run of 64 x 16 bytes. Work items (class, slab of P
//      positions, 16 blocks) go to per-XCD queues by slab, so one XCD
//      reads all blocks of a class at the same positions while their lines
//      are in its L2. Pass B adds the partial product and applies the
//      caller's epilogue (w = c1 H v + c2 u, raw output, accumulation).
#include "kern_common.h"

namespace hphi {

constexpr int kSplitBlocksPerItem = 16;   // one block per wave of a 1024-thread workgroup

struct SplitKArgs {
    const uint32_t *hi_list;       // high patterns by class, ascending
    const uint32_t *cls_first;     // n_hi + 2: class k's patterns at [cls_first[k], cls_first[k + 1])
    const uint64_t *hi_off;        // 2^n_hi + 1
    const HiBondDev *hib;
    int nhb;
    int n_lo, n_pop, P, lps;
    const uint32_t *cls_len;       // n_hi + 1: block length of class k
    const uint32_t *xcd_items;     // 8 x (n_hi + 2): per-XCD cumulative item counts by class
    int ncls;                      // n_hi + 1
    unsigned *sched;               // 8 queue counters + completion counter
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    void *raw_out;
    const double *coef;
    int coef_cplx;
};

__device__ __forceinline__ int split_xcc_id() { return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7u); }

template <typename S, int VPT>
__device__ __forceinline__ void ld_vpt(const S *p, S (&o)[VPT])
{
    if constexpr (VPT * sizeof(S) == 16) {
        const float4 t = *reinterpret_cast<const float4 *>(p);
        __builtin_memcpy(o, &t, 16);
    } else if constexpr (VPT * sizeof(S) == 8) {
        const float2 t = *reinterpret_cast<const float2 *>(p);
        __builtin_memcpy(o, &t, 8);
    } else {
#pragma unroll
        for (int j = 0; j < VPT; ++j) o[j] = p[j];
    }
}

// The same 16 bytes through non-temporal loads and stores: the streams of
// the partial product, u and the output are touched once and kept out of
// the way of the class slab in L2.
typedef float f4v __attribute__((ext_vector_type(4)));
template <typename S, int VPT>
__device__ __forceinline__ void ld_vpt_nt(const S *p, S (&o)[VPT])
{
    if constexpr (VPT * sizeof(S) == 16) {
        const f4v t = __builtin_nontemporal_load(reinterpret_cast<const f4v *>(p));
        __builtin_memcpy(o, &t, 16);
    } else {
#pragma unroll
        for (int j = 0; j < VPT; ++j) o[j] = __builtin_nontemporal_load(p + j);
    }
}
template <typename S, int VPT>
__device__ __forceinline__ void st_vpt_nt(S *p, const S (&o)[VPT])
{
    if constexpr (VPT * sizeof(S) == 16) {
        f4v t;
        __builtin_memcpy(&t, o, 16);
        __builtin_nontemporal_store(t, reinterpret_cast<f4v *>(p));
    } else {
#pragma unroll
        for (int j = 0; j < VPT; ++j) __builtin_nontemporal_store(o[j], p + j);
    }
}

template <typename S, int NV>
__global__ __launch_bounds__(1024) void k_spin_hi_pass(SplitKArgs a)
{
    constexpr int VPT = (NV * (int)sizeof(S) >= 16) ? 16 / (int)sizeof(S) : NV;
    typedef const __attribute__((address_space(4))) uint64_t CU64;
    __shared__ int s_item[3];
    __shared__ unsigned s_last;
    __shared__ HiBondDev s_hib[kMaxHiBonds];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int k = tid; k < a.nhb; k += blockDim.x) s_hib[k] = a.hib[k];
    // the table is read-only here: scalar loads at wave-uniform indices
    const CU64 *hoff = (const CU64 *)(a.hi_off);
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *accp = static_cast<S *>(a.acc_out);
    S *rawp = static_cast<S *>(a.raw_out);
    const S c1s = a.coef ? (S)a.coef[0] : (S)1, c2s = a.coef ? (S)a.coef[1] : (S)0;
    const int sub = lane % a.lps, pl = lane / a.lps;
    const int home = split_xcc_id();
    int q = home, tries = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            int k = -1, s = 0, g = 0;
            while (tries < 8) {
                const uint32_t *cum = a.xcd_items + q * (a.ncls + 1);
                const unsigned tot = cum[a.ncls];
                const unsigned i = atomicAdd(&a.sched[q], 1u);
                if (i < tot) {
                    int c = 0;
                    while (cum[c + 1] <= i) ++c;
                    const unsigned li = i - cum[c];
                    const unsigned ng = (a.cls_first[c + 1] - a.cls_first[c] + kSplitBlocksPerItem - 1) /
                                        kSplitBlocksPerItem;
                    k = c;
                    s = q + 8 * (int)(li / ng);
                    g = (int)(li % ng);
                    break;
                }
                q = (q + 1) & 7;
                ++tries;
            }
            s_item[0] = k;
            s_item[1] = s;
            s_item[2] = g;
        }
        __syncthreads();
        const int k = s_item[0];
        if (k < 0) break;
        const int slab = s_item[1];
        const uint32_t nblk = a.cls_first[k + 1] - a.cls_first[k];
        const uint32_t bi = (uint32_t)s_item[2] * kSplitBlocksPerItem + (uint32_t)wv;
        if (bi >= nblk) continue;
        const uint32_t h = __builtin_amdgcn_readfirstlane(a.hi_list[a.cls_first[k] + bi]);
        const uint64_t base = hoff[h];
        const int64_t p = (int64_t)slab * a.P + pl;
        const bool ok = p < (int64_t)a.cls_len[k];
        const size_t me = ((size_t)(base + p) * NV + (size_t)sub * VPT);
        S acc[VPT];
#pragma unroll
        for (int j = 0; j < VPT; ++j) acc[j] = (S)0;
        double dg = 0.0;
        // high bonds in batches of eight: targets (wave-uniform) first, then
        // the eight contiguous gathers in flight, then the sums in bond order
        for (int b0 = 0; b0 < a.nhb; b0 += 8) {
            uint64_t src[8];
            S cf[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                src[t] = base;
                cf[t] = (S)0;
                if (b0 + t < a.nhb) {
                    const HiBondDev bd = s_hib[b0 + t];
                    const uint32_t mk = __builtin_amdgcn_readfirstlane(bd.mask);
                    const uint32_t tb = h & mk;
                    if (tb == 0u || tb == mk) {
                        dg += bd.jz4;
                    } else {
                        dg -= bd.jz4;
                        src[t] = hoff[h ^ mk];
                        cf[t] = (S)bd.jxy2;
                    }
                }
            }
            S g[8][VPT];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                if (ok) ld_vpt<S, VPT>(v + (size_t)(src[t] + p) * NV + (size_t)sub * VPT, g[t]);
                else {
#pragma unroll
                    for (int j = 0; j < VPT; ++j) g[t][j] = (S)0;
                }
            }
#pragma unroll
            for (int t = 0; t < 8; ++t)
#pragma unroll
                for (int j = 0; j < VPT; ++j) acc[j] += cf[t] * g[t][j];
        }
        if (!ok) continue;
        S me_v[VPT], wp[VPT], hv[VPT], out[VPT];
        ld_vpt<S, VPT>(v + me, me_v);
        ld_vpt_nt<S, VPT>(w + me, wp);
#pragma unroll
        for (int j = 0; j < VPT; ++j) hv[j] = wp[j] + acc[j] + (S)dg * me_v[j];
        if (a.coef_cplx) {
            S uu[VPT];
#pragma unroll
            for (int j = 0; j < VPT; ++j) uu[j] = (S)0;
            if (u) ld_vpt_nt<S, VPT>(u + me, uu);
            epilogue_r<S, VPT>(hv, uu, u != nullptr, 1, a.coef, out);
        } else {
            S uu[VPT];
            if (u) ld_vpt_nt<S, VPT>(u + me, uu);
#pragma unroll
            for (int j = 0; j < VPT; ++j) out[j] = c1s * hv[j] + (u ? c2s * uu[j] : (S)0);
        }
        st_vpt_nt<S, VPT>(w + me, out);
        if (rawp) {
#pragma unroll
            for (int j = 0; j < VPT; ++j) rawp[me + j] = hv[j];
        }
        if (accp) {
#pragma unroll
            for (int j = 0; j < VPT; ++j) accp[me + j] += out[j];
        }
    }
    // the last workgroup re-arms the queues for the next launch
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        s_last = (atomicAdd(&a.sched[8], 1u) == gridDim.x - 1) ? 1u : 0u;
        if (s_last) {
            for (int i = 0; i < 9; ++i) a.sched[i] = 0u;
            __threadfence();
        }
    }
}

// Host tables: the high bonds, the other bonds, the high patterns by
// class, and per (positions per wave) the per-XCD cumulative item counts.
int spin_split_tables(hphi_ham *h)
{
    if (h->split.built) return HPHI_OK;
    const Species &s = h->basis->sp[0];
    const int n_lo = s.n_lo;
    std::vector<HiBondDev> hi;
    std::vector<SpinBondDev> rest;
    for (const SpinBondDev &b : h->bonds) {
        if (b.i >= n_lo && b.j >= n_lo) {
            HiBondDev d{};
            d.mask = (uint32_t)(b.mask >> n_lo);
            d.jz4 = b.jz4;
            d.jxy2 = b.jxy2;
            hi.push_back(d);
        } else {
            rest.push_back(b);
        }
    }
    h->split.n_hi_bonds = (int)hi.size();
    h->split.n_rest = (int)rest.size();
    if (hi.empty()) hi.push_back(HiBondDev{});
    if (rest.empty()) rest.push_back(SpinBondDev{});
    HPHI_TRY(upload(h->split.hib, hi.data(), sizeof(HiBondDev) * hi.size()));
    HPHI_TRY(upload(h->split.rest, rest.data(), sizeof(SpinBondDev) * rest.size()));
    const int n_hi = s.n_hi;
    std::vector<uint32_t> first(n_hi + 2, 0), list;
    std::vector<std::vector<uint32_t>> by(n_hi + 1);
    for (uint32_t x = 0; x < (1u << n_hi); ++x) by[__builtin_popcount(x)].push_back(x);
    std::vector<uint32_t> len(n_hi + 1, 0);
    for (int k = 0; k <= n_hi; ++k) {
        first[k] = (uint32_t)list.size();
        const int need = s.n_pop - k;
        if (need >= 0 && need <= n_lo) {
            list.insert(list.end(), by[k].begin(), by[k].end());
            uint64_t c = 1;
            for (int t = 1; t <= need; ++t) c = c * (uint64_t)(n_lo - need + t) / (uint64_t)t;
            len[k] = (uint32_t)c;
        }
    }
    first[n_hi + 1] = (uint32_t)list.size();
    if (list.empty()) list.push_back(0);
    HPHI_TRY(upload(h->split.hi_list, list.data(), sizeof(uint32_t) * list.size()));
    HPHI_TRY(upload(h->split.cls_first, first.data(), sizeof(uint32_t) * first.size()));
    HPHI_TRY(upload(h->split.cls_len, len.data(), sizeof(uint32_t) * len.size()));
    h->split.cls_first_h = first;
    h->split.cls_len_h = len;
    h->split.built = true;
    return HPHI_OK;
}

static int split_items(hphi_ham *h, int P)
{
    const int pi = __builtin_ctz((unsigned)P);
    if (h->split.items_ok[pi]) return HPHI_OK;
    const int n_hi = h->basis->sp[0].n_hi, ncls = n_hi + 1;
    std::vector<uint32_t> cum(8 * (ncls + 1), 0);
    for (int x = 0; x < 8; ++x) {
        uint32_t acc = 0;
        for (int k = 0; k < ncls; ++k) {
            cum[x * (ncls + 1) + k] = acc;
            const uint32_t nb = h->split.cls_first_h[k + 1] - h->split.cls_first_h[k];
            const uint32_t L = h->split.cls_len_h[k];
            if (nb == 0 || L == 0) continue;
            const uint32_t nsl = (L + P - 1) / P;
            const uint32_t mine = nsl > (uint32_t)x ? (nsl - x + 7) / 8 : 0;
            const uint32_t ng = (nb + kSplitBlocksPerItem - 1) / kSplitBlocksPerItem;
            const uint64_t add = (uint64_t)mine * ng;
            if (acc + add >= (1ull << 31)) return fail(HPHI_ERR_UNSUPPORTED, "split spin H*v: too many work items");
            acc += (uint32_t)add;
        }
        cum[x * (ncls + 1) + ncls] = acc;
    }
    HPHI_TRY(upload(h->split.items[pi], cum.data(), sizeof(uint32_t) * cum.size()));
    h->split.items_ok[pi] = true;
    return HPHI_OK;
}

template <typename S, int NV>
static int launch_hi_t(hphi_ham *h, const MultArgs &m)
{
    constexpr int VPT = (NV * (int)sizeof(S) >= 16) ? 16 / (int)sizeof(S) : NV;
    constexpr int LPS = NV / VPT;
    static_assert(LPS >= 1 && LPS <= 64, "lanes per state");
    const int P = 64 / LPS;
    HPHI_TRY(split_items(h, P));
    const Species &s = h->basis->sp[0];
    SplitKArgs a{};
    a.hi_list = h->split.hi_list.as<uint32_t>();
    a.cls_first = h->split.cls_first.as<uint32_t>();
    a.hi_off = s.d_hi_off.as<uint64_t>();
    a.hib = h->split.hib.as<HiBondDev>();
    a.nhb = h->split.n_hi_bonds;
    a.n_lo = s.n_lo;
    a.n_pop = s.n_pop;
    a.P = P;
    a.lps = LPS;
    a.cls_len = h->split.cls_len.as<uint32_t>();
    a.xcd_items = h->split.items[__builtin_ctz((unsigned)P)].as<uint32_t>();
    a.ncls = s.n_hi + 1;
    a.sched = h->sched.as<unsigned>();
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.raw_out = m.raw_out;
    a.coef = m.coef;
    a.coef_cplx = m.coef_cplx;
    const int ncu = h->basis->ctx->n_cu > 0 ? h->basis->ctx->n_cu : 256;
    hipLaunchKernelGGL((k_spin_hi_pass<S, NV>), dim3(2 * ncu), dim3(1024), 0, m.stream, a);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_spin_hi_pass(hphi_ham *h, const MultArgs &m)
{
    const int nv = m.nvec * dtype_lanes(m.dtype);
    const bool f32 = dtype_is_f32(m.dtype);
    switch (nv) {
    case 1: return f32 ? launch_hi_t<float, 1>(h, m) : launch_hi_t<double, 1>(h, m);
    case 2: return f32 ? launch_hi_t<float, 2>(h, m) : launch_hi_t<double, 2>(h, m);
    case 4: return f32 ? launch_hi_t<float, 4>(h, m) : launch_hi_t<double, 4>(h, m);
    case 8: return f32 ? launch_hi_t<float, 8>(h, m) : launch_hi_t<double, 8>(h, m);
    case 16: return f32 ? launch_hi_t<float, 16>(h, m) : launch_hi_t<double, 16>(h, m);
    case 32: return f32 ? launch_hi_t<float, 32>(h, m) : launch_hi_t<double, 32>(h, m);
    }
    return fail(HPHI_ERR_UNSUPPORTED, "split spin H*v: %d lanes", nv);
}

} // namespace hphi

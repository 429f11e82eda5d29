// Two-body terms of the general Hubbard Hamiltonian (HPhi update paper
// Sec. 5, Eq. ham_general), per site pair p = (i, j), M = {i, j}:
//   V n_i n_j - JH (n_i,up n_j,up + n_i,dn n_j,dn)
//   + JX (c+_i,up c_j,up c+_j,dn c_i,dn + h.c.)    exchange
//   + JP (c+_i,up c_j,up c+_i,dn c_j,dn + h.c.)    pair hopping
// Both off-diagonal kinds move one up and one down electron across the
// pair: (u, d) -> (u ^ M, d ^ M), allowed when u and d each hold exactly one
// electron on M. Both on the same site: pair hopping; on different sites:
// exchange. With all up orbitals ordered before all down orbitals each
// product is an up bilinear times a down bilinear, so the element is
// J (-1)^(up sites strictly between i and j) (-1)^(down sites between).
// The diagonal splits into E_up(u) + E_dn(d) + sum_{k in d} m_k(u): the
// same-species parts (V - JH) u_i u_j and (V - JH) d_i d_j from tables, the
// cross part V (u_i d_j + d_i u_j) from per-row site weights m_k(u).
//
// One workgroup per up row (grid-stride). The row-uniform work -- the pairs
// that can act on this u, their target up row and up sign, and byte tables
// of the site weights (sum over the set bits of one byte of d) -- is done
// once per row in LDS; the lanes then run over the down states, gather the
// targets (down rank from the species' two-level table) and add into w.
// The product runs between the T_dn/U rows kernel and the T_up kernel, so
// the latter's fused epilogue and dot products see the whole H*v.
#include "kern_common.h"

namespace hphi {

struct PairKArgs {
    const uint32_t *ups, *dns;
    int64_t dup, ddn, ld;
    const HubPairDev *pairs;
    int np;
    const double *eup, *edn;
    const uint32_t *site_off;
    const PairNbrDev *site_nbr;
    const uint32_t *hi_off_up, *lo_rank_up, *hi_off_dn, *lo_rank_dn;
    int nlo_up, nlo_dn;
    int n_sites;
    const void *v;
    void *w;
};

// RANK_LDS: the down species' rank tables copied into dynamic LDS (they are
// 2^n_hi + 1 + 2^n_lo words: 2 KB at 16 sites)
template <typename S, int NV, bool RANK_LDS>
__global__ __launch_bounds__(1024) void k_hub_pairs(PairKArgs a)
{
    // active pairs of the current row, in pair order
    __shared__ uint32_t s_mask[kMaxPairTerms], s_bw[kMaxPairTerms], s_um[kMaxPairTerms];
    __shared__ int64_t s_off[kMaxPairTerms];            // target up row * ld
    __shared__ double s_jx[kMaxPairTerms], s_jp[kMaxPairTerms];   // up sign folded in
    __shared__ double s_m[32];                          // cross weights m_k(u)
    __shared__ double s_bt[4][256];                     // byte tables of m
    __shared__ uint32_t s_cnt;
    extern __shared__ uint32_t s_rank[];
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const int tid = threadIdx.x, T = blockDim.x;
    const int nchunk = (a.n_sites + 7) >> 3;
    const uint32_t lomask_up = (1u << a.nlo_up) - 1u, lomask_dn = (1u << a.nlo_dn) - 1u;
    const int nhi_dn = a.n_sites - a.nlo_dn;
    const uint32_t *hi_dn = a.hi_off_dn, *lo_dn = a.lo_rank_dn;
    if constexpr (RANK_LDS) {
        const int nh = (1 << nhi_dn) + 1, nl = 1 << a.nlo_dn;
        for (int k = tid; k < nh; k += T) s_rank[k] = a.hi_off_dn[k];
        for (int k = tid; k < nl; k += T) s_rank[nh + k] = a.lo_rank_dn[k];
        hi_dn = s_rank;
        lo_dn = s_rank + nh;
    }
    for (int64_t ru = blockIdx.x; ru < a.dup; ru += gridDim.x) {
        const uint32_t u = a.ups[ru];
        __syncthreads();   // the previous row's tables are no longer read
        if (tid < 64) {
            // wave 0 compacts the pairs that can act on u (order kept)
            uint32_t base = 0;
            for (int p0 = 0; p0 < a.np; p0 += 64) {
                const int p = p0 + tid;
                bool act = false;
                HubPairDev q{};
                if (p < a.np) {
                    q = a.pairs[p];
                    act = __builtin_popcount(u & q.mask) == 1 && (q.jx != 0.0 || q.jp != 0.0);
                }
                const uint64_t bal = __ballot(act);
                if (act) {
                    const uint32_t pos = base + (uint32_t)__builtin_popcountll(bal & ((1ull << tid) - 1ull));
                    const uint32_t u2 = u ^ q.mask;
                    const int64_t r2 = (int64_t)a.hi_off_up[u2 >> a.nlo_up] + a.lo_rank_up[u2 & lomask_up];
                    const double su = (__builtin_popcount(u & q.between) & 1) ? -1.0 : 1.0;
                    s_mask[pos] = q.mask;
                    s_bw[pos] = q.between;
                    s_um[pos] = u & q.mask;
                    s_off[pos] = r2 * a.ld;
                    s_jx[pos] = su * q.jx;
                    s_jp[pos] = su * q.jp;
                }
                base += (uint32_t)__builtin_popcountll(bal);
            }
            if (tid == 0) s_cnt = base;
        } else if (tid - 64 < a.n_sites) {
            const int k = tid - 64;
            double m = 0.0;
            for (uint32_t e = a.site_off[k]; e < a.site_off[k + 1]; ++e)
                m += a.site_nbr[e].v * (double)((u >> a.site_nbr[e].other) & 1u);
            s_m[k] = m;
        }
        __syncthreads();
        for (int e = tid; e < nchunk * 256; e += T) {
            const int c = e >> 8, b = e & 255;
            double s = 0.0;
            for (int q = 0; q < 8; ++q)
                if (((b >> q) & 1) && 8 * c + q < a.n_sites) s += s_m[8 * c + q];
            s_bt[c][b] = s;
        }
        __syncthreads();
        const uint32_t cnt = s_cnt;
        const double eu = a.eup[ru];
        for (int64_t rd = tid; rd < a.ddn; rd += T) {
            const uint32_t d = a.dns[rd];
            double dg = eu + a.edn[rd];
            for (int c = 0; c < nchunk; ++c) dg += s_bt[c][(d >> (8 * c)) & 255u];
            const size_t me = ((size_t)ru * a.ld + rd) * NV;
            double acc[NV];
#pragma unroll
            for (int l = 0; l < NV; ++l) acc[l] = dg * (double)v[me + l];
            // active pairs in batches of eight: targets and coefficients
            // first, then all eight gathers in flight, then the sums in
            // pair order (an inactive slot adds 0 x v[me])
            constexpr int B = 8;
            for (uint32_t k0 = 0; k0 < cnt; k0 += B) {
                size_t src[B];
                double cf[B];
#pragma unroll
                for (int t = 0; t < B; ++t) {
                    const uint32_t k = k0 + t;
                    src[t] = me;
                    cf[t] = 0.0;
                    if (k < cnt) {
                        const uint32_t mk = s_mask[k];
                        const uint32_t dm = d & mk;
                        if (__builtin_popcount(dm) == 1) {
                            const double c = dm == s_um[k] ? s_jp[k] : s_jx[k];
                            const uint32_t d2 = d ^ mk;
                            const int64_t r2 = (int64_t)hi_dn[d2 >> a.nlo_dn] + lo_dn[d2 & lomask_dn];
                            cf[t] = (__builtin_popcount(d & s_bw[k]) & 1) ? -c : c;
                            src[t] = (size_t)(s_off[k] + r2) * NV;
                        }
                    }
                }
                S g[B][NV];
#pragma unroll
                for (int t = 0; t < B; ++t)
#pragma unroll
                    for (int l = 0; l < NV; ++l) g[t][l] = v[src[t] + l];
#pragma unroll
                for (int t = 0; t < B; ++t)
#pragma unroll
                    for (int l = 0; l < NV; ++l) acc[l] += cf[t] * (double)g[t][l];
            }
#pragma unroll
            for (int l = 0; l < NV; ++l) w[me + l] += (S)acc[l];
        }
    }
}

int launch_hub_pairs(hphi_ham *h, int elem_bytes, int nv, const void *v, void *w, int64_t ld, hipStream_t st)
{
    if (h->kind != 1 || h->hub.n_pairs == 0) return HPHI_OK;
    const hphi_basis *b = h->basis;
    const Species &up = b->sp[0], &dn = b->sp[1];
    if (!up.d_hi_off32.p || !dn.d_hi_off32.p || b->n_sites > 32)
        return fail(HPHI_ERR_UNSUPPORTED, "two-body terms need 32-bit species rank tables");
    PairKArgs a{};
    a.ups = up.d_states.as<uint32_t>();
    a.dns = dn.d_states.as<uint32_t>();
    a.dup = up.dim;
    a.ddn = dn.dim;
    a.ld = ld > 0 ? ld : dn.dim;
    a.pairs = h->hub.pairs.as<HubPairDev>();
    a.np = h->hub.n_pairs;
    a.eup = h->hub.pair_eup.as<double>();
    a.edn = h->hub.pair_edn.as<double>();
    a.site_off = h->hub.pair_site_off.as<uint32_t>();
    a.site_nbr = h->hub.pair_site_nbr.as<PairNbrDev>();
    a.hi_off_up = up.d_hi_off32.as<uint32_t>();
    a.lo_rank_up = up.d_lo_rank.as<uint32_t>();
    a.hi_off_dn = dn.d_hi_off32.as<uint32_t>();
    a.lo_rank_dn = dn.d_lo_rank.as<uint32_t>();
    a.nlo_up = up.n_lo;
    a.nlo_dn = dn.n_lo;
    a.n_sites = b->n_sites;
    a.v = v;
    a.w = w;
    const int ncu = b->ctx->n_cu > 0 ? b->ctx->n_cu : 256;
    const unsigned grid = (unsigned)std::min<int64_t>(a.dup, 2 * (int64_t)ncu);
    const size_t rank_words = ((size_t)1 << (b->n_sites - dn.n_lo)) + 1 + ((size_t)1 << dn.n_lo);
    const bool rank_lds = rank_words * 4 <= 32 * 1024;
    const size_t lds = rank_lds ? rank_words * 4 : 0;
    auto go = [&](auto kern) {
        hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(1024), lds, st, a);
    };
    if (elem_bytes == 8 && nv == 1) rank_lds ? go(k_hub_pairs<double, 1, true>) : go(k_hub_pairs<double, 1, false>);
    else if (elem_bytes == 8 && nv == 2) rank_lds ? go(k_hub_pairs<double, 2, true>) : go(k_hub_pairs<double, 2, false>);
    else if (elem_bytes == 4 && nv == 1) rank_lds ? go(k_hub_pairs<float, 1, true>) : go(k_hub_pairs<float, 1, false>);
    else if (elem_bytes == 4 && nv == 2) rank_lds ? go(k_hub_pairs<float, 2, true>) : go(k_hub_pairs<float, 2, false>);
    else return fail(HPHI_ERR_UNSUPPORTED, "two-body terms: %d-byte elements, %d lanes", elem_bytes, nv);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

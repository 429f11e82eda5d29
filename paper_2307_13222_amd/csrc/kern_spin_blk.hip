// Spin-1/2 XXZ H*v one block of states at a time (HPhi update paper Sec.
// 3.2 Heisenberg model; the Lanczos runs on sectors of about 10^10 states
// that motivate Sec. 1, and the cTPQ blocks of Sec. 3.5.1). It needs no
// stored state list: the default on the implicit basis, and a schedule
// choice on the stored one.
//
// A split point n_lo of the sites (chosen so that a block fits LDS; it need
// not be the basis's own) cuts a state x into (h, l). The basis order is
// ascending x whatever the split, so the states of one high pattern h form
// a block in ascending l, the state (h, l) at hi_off[h] + lo_rank[l] with
// the tables of this split point. A workgroup takes one block at a time:
//   * it stages the block's values in LDS (one contiguous read);
//   * a bond inside the low part maps position p to a position q of the
//     same block; q comes from a per-bond table over the low patterns, read
//     contiguously along p, and the partner value from LDS;
//   * a bond inside the high part maps (h, p) to (h ^ m, p): the partner
//     block's start is the same for the whole workgroup and the lanes read
//     consecutive positions of it;
//   * a bond with one end in each part flips one low site and one high
//     site: the partner block is again common to the workgroup, the partner
//     position comes from a per-site table over the low patterns, and the
//     lanes' partner positions ascend with p.
// No configuration is unranked and no rank table is searched per flip. The
// caller's epilogue (w = c1 H v + c2 u with real or complex coefficients,
// accumulation, the raw product) is applied at the end. Sums are in bond
// order within each kind (low, crossing, high), so they equal the one-pass
// products up to summation order.
#include "kern_common.h"

#include <algorithm>

namespace hphi {

namespace {

struct BlkKArgs {
    const uint32_t *hi_list;   // the high patterns with a nonempty block, by popcount
    uint32_t n_blocks;
    const uint64_t *hi_off;    // 2^n_hi + 1
    const uint32_t *lo_list;   // low patterns grouped by popcount
    const uint32_t *cls_len;   // by popcount of h: block length
    const uint32_t *lo_off;    // by popcount of h: first lo_list index of its low patterns
    const LoBondDev *lob;
    const XBondDev *xb;
    const HiBondDev *hib;
    int nlob, nxb, nhib;
    const uint16_t *tab;       // rows of 2^n_lo partner positions
    uint64_t pitch;            // 2^n_lo
    const double *hz;          // per site or null
    int n_lo, n_sites;
    unsigned *sched;           // [0] block counter, [1] finished workgroups
    const void *v;
    void *w;
    const void *u;
    void *acc_out;
    const double *coef;
    void *raw_out;       // several lanes per state: H v before the epilogue (optional)
    int coef_cplx;       // several lanes per state: complex (c1, c2) on lane pairs
};

// Occupancy, not the block size, sets the pace (each position waits on
// chains of table loads, LDS reads and gathers): 512-thread workgroups,
// four per CU for FP32 values (eight waves per SIMD), 256-thread
// workgroups, five per CU, for FP64 values (more registers per lane);
// the split point is chosen so that a block leaves room for that many
// (36-site J1-J2 sector: FP32 H*v 1.17 s with one 1024-thread workgroup
// per CU and blocks of 17 low sites, 0.89 s with three of 512 and 16 low
// sites, 0.81 s with four of 512 and 15 low sites; FP64 1.35 s against
// 1.20 s with five of 256 and 14 low sites). FP32 states of several lanes
// (blocks of vectors) also take four 512-thread workgroups at eight waves
// per SIMD, with a few registers spilled (28-site block of 16 complex64
// vectors: 17.6 ms with blocks of 10 low sites; 19.6 ms with 11 low sites
// and two per CU at five waves per SIMD, 22.2 ms with 10 low sites there,
// 31.1 ms with 12 and one per CU); FP64 ones two per CU.
constexpr int kBlkMaxThreads = 512;
constexpr int kBatch = 16;
constexpr size_t kCuLds = 160 * 1024;
int blk_threads(int esize, bool f32) { return !f32 && esize == 8 ? 256 : 512; }
int blk_per_cu(int esize, bool f32) { return f32 ? 4 : esize == 8 ? 5 : 2; }

// 4-byte values: registers held to 64 VGPRs and the scalar registers of
// eight waves per SIMD (no spills), so four 512-thread workgroups share a CU
template <typename S>
__global__ __launch_bounds__(kBlkMaxThreads) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 4 ? 8 : 1, 8)))
void k_spin_blk(BlkKArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *blk = reinterpret_cast<S *>(smem_raw);
    __shared__ unsigned s_i;
    __shared__ unsigned s_last;
    // the block's flipping high bonds, in bond order: partner block start
    // and coefficient (the flips depend on h only)
    __shared__ uint64_t s_hsrc[kMaxHiBonds];
    __shared__ S s_hcf[kMaxHiBonds];
    __shared__ unsigned s_wn[kMaxHiBonds / 64];
    __shared__ uint64_t s_xpb[kMaxHiBonds];   // crossing bond b: its partner block's start
    // read-only tables at workgroup-uniform indices: scalar loads
    typedef const __attribute__((address_space(4))) uint64_t CU64;
    typedef const __attribute__((address_space(4))) uint32_t CU32;
    typedef const __attribute__((address_space(4))) LoBondDev CLB;
    typedef const __attribute__((address_space(4))) XBondDev CXB;
    typedef const __attribute__((address_space(4))) HiBondDev CHB;
    const CU64 *hoff = (const CU64 *)a.hi_off;
    const CU32 *hlist = (const CU32 *)a.hi_list;
    const CU32 *clen = (const CU32 *)a.cls_len;
    const CU32 *loff = (const CU32 *)a.lo_off;
    const CLB *lob = (const CLB *)a.lob;
    const CXB *xb = (const CXB *)a.xb;
    const CHB *hib = (const CHB *)a.hib;
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *__restrict__ accp = static_cast<S *>(a.acc_out);
    const uint16_t *__restrict__ tab = a.tab;
    const uint32_t *__restrict__ lol = a.lo_list;
    const S c1s = a.coef ? (S)a.coef[0] : (S)1, c2s = a.coef ? (S)a.coef[1] : (S)0;
    const int tid = threadIdx.x;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_i = atomicAdd(&a.sched[0], 1u);
        __syncthreads();
        const unsigned bi = __builtin_amdgcn_readfirstlane(s_i);
        if (bi >= a.n_blocks) break;
        const uint32_t hh = hlist[bi];
        const int k = __builtin_popcount(hh);
        const uint32_t L = clen[k];
        const uint32_t g0 = loff[k];
        const uint64_t base = hoff[hh];
        // stage the block: four loads in flight per thread
        const uint32_t nt = blockDim.x;
        for (uint32_t p0 = tid; p0 < L; p0 += 4 * nt) {
            S t[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t p = p0 + (uint32_t)r * nt;
                t[r] = p < L ? v[base + p] : (S)0;
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t p = p0 + (uint32_t)r * nt;
                if (p < L) blk[p] = t[r];
            }
        }
        __syncthreads();
        // the high bonds' diagonal and the high sites' fields: the same for
        // every state of the block
        {
            const int i = tid;
            bool f = false;
            uint32_t mk = 0u;
            if (i < a.nhib) {
                mk = a.hib[i].mask;
                const uint32_t tt = hh & mk;
                f = tt != 0u && tt != mk;
            }
            const uint64_t bal = __ballot(f);
            const int lane = tid & 63;
            if (i < kMaxHiBonds && lane == 0) s_wn[i >> 6] = (unsigned)__popcll(bal);
            __syncthreads();
            if (f) {
                unsigned at = (unsigned)__popcll(bal & ((uint64_t(1) << lane) - 1));
                for (int w = 0; w < (i >> 6); ++w) at += s_wn[w];
                s_hsrc[at] = a.hi_off[hh ^ mk];
                s_hcf[at] = (S)a.hib[i].jxy2;
            }
            // (FP32 only: with FP64 values the extra registers cost a wave)
            if constexpr (sizeof(S) == 4)
                if (i < a.nxb) s_xpb[i] = a.hi_off[hh ^ (1u << a.xb[i].hbit)];
            __syncthreads();
        }
        int nha = 0;
        for (int w = 0; w < (a.nhib + 63) / 64; ++w) nha += (int)s_wn[w];
        S dgh = (S)0;
        for (int b = 0; b < a.nhib; ++b) {
            const uint32_t mk = hib[b].mask;
            const uint32_t t = hh & mk;
            dgh += (t == 0u || t == mk) ? (S)hib[b].jz4 : -(S)hib[b].jz4;
        }
        if (a.hz)
            for (int i = a.n_lo; i < a.n_sites; ++i)
                dgh -= (S)a.hz[i] * (((hh >> (i - a.n_lo)) & 1u) ? (S)0.5 : (S)-0.5);
        for (uint32_t p = tid; p < L; p += nt) {
            const uint32_t g = g0 + p;
            const uint32_t l = lol[g];
            S acc = (S)0, dg = dgh;
            if (a.hz)
                for (int i = 0; i < a.n_lo; ++i) dg -= (S)a.hz[i] * (((l >> i) & 1u) ? (S)0.5 : (S)-0.5);
            // bonds inside the low part: partners in LDS
            for (int b0 = 0; b0 < a.nlob; b0 += kBatch) {
                uint32_t q[kBatch];
                S cf[kBatch];
                unsigned anti = 0u;
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    q[t] = 0u;
                    cf[t] = (S)0;
                    const int b = b0 + t;
                    if (b < a.nlob) {
                        const uint32_t mk = lob[b].mask;
                        const uint32_t tt = l & mk;
                        const S jz = (S)lob[b].jz4;
                        if (tt == 0u || tt == mk) {
                            dg += jz;
                        } else {
                            dg -= jz;
                            anti |= 1u << t;
                            cf[t] = (S)lob[b].jxy2;
                        }
                        q[t] = tab[(uint64_t)lob[b].row * a.pitch + g];
                    }
                }
#pragma unroll
                for (int t = 0; t < kBatch; ++t)
                    if (anti & (1u << t)) acc += cf[t] * blk[q[t]];
            }
            // bonds across the split: one position of a partner block
            for (int b0 = 0; b0 < a.nxb; b0 += kBatch) {
                uint64_t src[kBatch];
                S cf[kBatch], val[kBatch];
                unsigned anti = 0u;
                uint32_t qlast = 0u, rlast = 0xffffffffu;
#pragma unroll
                for (int t = 0; t < kBatch; ++t) {
                    src[t] = 0;
                    cf[t] = (S)0;
                    const int b = b0 + t;
                    if (b < a.nxb) {
                        const uint32_t hbit = xb[b].hbit;
                        uint64_t pb;
                        if constexpr (sizeof(S) == 4) pb = s_xpb[b];
                        else pb = hoff[hh ^ (1u << hbit)];
                        const uint32_t row = xb[b].row;
                        if (row != rlast) {
                            qlast = tab[(uint64_t)row * a.pitch + g];
                            rlast = row;
                        }
                        const uint32_t q = qlast;
                        const uint32_t hb = (hh >> hbit) & 1u;
                        const uint32_t lb = (l >> xb[b].lbit) & 1u;
                        const S jz = (S)xb[b].jz4;
                        if (hb == lb) {
                            dg += jz;
                        } else {
                            dg -= jz;
                            anti |= 1u << t;
                            cf[t] = (S)xb[b].jxy2;
                            src[t] = pb + q;
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < kBatch; ++t) val[t] = (anti & (1u << t)) ? v[src[t]] : (S)0;
#pragma unroll
                for (int t = 0; t < kBatch; ++t)
                    if (anti & (1u << t)) acc += cf[t] * val[t];
            }
            // bonds inside the high part: the same position of a partner
            // block, the block's flipping ones only
            for (int b0 = 0; b0 < nha; b0 += kBatch) {
                S val[kBatch];
#pragma unroll
                for (int t = 0; t < kBatch; ++t) val[t] = b0 + t < nha ? v[s_hsrc[b0 + t] + p] : (S)0;
#pragma unroll
                for (int t = 0; t < kBatch; ++t)
                    if (b0 + t < nha) acc += s_hcf[b0 + t] * val[t];
            }
            const S hv = acc + dg * blk[p];
            S out = c1s * hv;
            if (u) out += c2s * u[base + p];
            w[base + p] = out;
            if (accp) accp[base + p] += out;
        }
    }
    // the last workgroup re-arms the counters for the next launch
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        s_last = (atomicAdd(&a.sched[1], 1u) == gridDim.x - 1) ? 1u : 0u;
        if (s_last) {
            a.sched[0] = 0u;
            a.sched[1] = 0u;
            __threadfence();
        }
    }
}

// Several real lanes per state (a block of vectors, complex vectors): the
// same walk with LPS lanes per state, each holding VPT consecutive values
// (16 bytes where the state has that many); the LDS block holds whole
// states, so every partner read is one 16-byte piece per lane.
constexpr int kBatchV = 8;

template <typename S, int VPT>
__device__ __forceinline__ void ld_piece(const S *p, S (&o)[VPT])
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
template <typename S, int VPT>
__device__ __forceinline__ void st_piece(S *p, const S (&o)[VPT])
{
    if constexpr (VPT * sizeof(S) == 16) {
        float4 t;
        __builtin_memcpy(&t, o, 16);
        *reinterpret_cast<float4 *>(p) = t;
    } else if constexpr (VPT * sizeof(S) == 8) {
        float2 t;
        __builtin_memcpy(&t, o, 8);
        *reinterpret_cast<float2 *>(p) = t;
    } else {
#pragma unroll
        for (int j = 0; j < VPT; ++j) p[j] = o[j];
    }
}

template <typename S, int NV>
__global__ __launch_bounds__(kBlkMaxThreads) __attribute__((amdgpu_waves_per_eu(sizeof(S) == 4 ? 8 : 1, 8)))
void k_spin_blk_v(BlkKArgs a)
{
    constexpr int VPT = (NV * (int)sizeof(S) >= 16) ? 16 / (int)sizeof(S) : NV;
    constexpr int LPS = NV / VPT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    S *blk = reinterpret_cast<S *>(smem_raw);
    __shared__ unsigned s_i;
    __shared__ unsigned s_last;
    __shared__ uint64_t s_hsrc[kMaxHiBonds];
    __shared__ S s_hcf[kMaxHiBonds];
    __shared__ unsigned s_wn[kMaxHiBonds / 64];
    typedef const __attribute__((address_space(4))) uint64_t CU64;
    typedef const __attribute__((address_space(4))) uint32_t CU32;
    typedef const __attribute__((address_space(4))) LoBondDev CLB;
    typedef const __attribute__((address_space(4))) XBondDev CXB;
    typedef const __attribute__((address_space(4))) HiBondDev CHB;
    const CU64 *hoff = (const CU64 *)a.hi_off;
    const CU32 *hlist = (const CU32 *)a.hi_list;
    const CU32 *clen = (const CU32 *)a.cls_len;
    const CU32 *loff = (const CU32 *)a.lo_off;
    const CLB *lob = (const CLB *)a.lob;
    const CXB *xb = (const CXB *)a.xb;
    const CHB *hib = (const CHB *)a.hib;
    const S *__restrict__ v = static_cast<const S *>(a.v);
    S *__restrict__ w = static_cast<S *>(a.w);
    const S *__restrict__ u = static_cast<const S *>(a.u);
    S *__restrict__ accp = static_cast<S *>(a.acc_out);
    S *__restrict__ rawp = static_cast<S *>(a.raw_out);
    const uint16_t *__restrict__ tab = a.tab;
    const uint32_t *__restrict__ lol = a.lo_list;
    const int tid = threadIdx.x, sub = tid % LPS;
    const uint32_t nt = blockDim.x, sp = nt / LPS, ps = (uint32_t)tid / LPS;
    for (;;) {
        __syncthreads();
        if (tid == 0) s_i = atomicAdd(&a.sched[0], 1u);
        __syncthreads();
        const unsigned bi = __builtin_amdgcn_readfirstlane(s_i);
        if (bi >= a.n_blocks) break;
        const uint32_t hh = hlist[bi];
        const int k = __builtin_popcount(hh);
        const uint32_t L = clen[k];
        const uint32_t g0 = loff[k];
        const uint64_t base = hoff[hh];
        // stage the block's states, VPT values per piece, four in flight
        const uint32_t npc = L * LPS;
        const S *vb = v + base * NV;
        for (uint32_t c0 = tid; c0 < npc; c0 += 4 * nt) {
            S t[4][VPT];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t c = c0 + (uint32_t)r * nt;
                if (c < npc) ld_piece<S, VPT>(vb + (size_t)c * VPT, t[r]);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const uint32_t c = c0 + (uint32_t)r * nt;
                if (c < npc) st_piece<S, VPT>(blk + (size_t)c * VPT, t[r]);
            }
        }
        __syncthreads();
        // the block's flipping high bonds, in bond order (as k_spin_blk)
        {
            const int i = tid;
            bool f = false;
            uint32_t mk = 0u;
            if (i < a.nhib) {
                mk = a.hib[i].mask;
                const uint32_t tt = hh & mk;
                f = tt != 0u && tt != mk;
            }
            const uint64_t bal = __ballot(f);
            const int lane = tid & 63;
            if (i < kMaxHiBonds && lane == 0) s_wn[i >> 6] = (unsigned)__popcll(bal);
            __syncthreads();
            if (f) {
                unsigned at = (unsigned)__popcll(bal & ((uint64_t(1) << lane) - 1));
                for (int w = 0; w < (i >> 6); ++w) at += s_wn[w];
                s_hsrc[at] = a.hi_off[hh ^ mk];
                s_hcf[at] = (S)a.hib[i].jxy2;
            }
            __syncthreads();
        }
        int nha = 0;
        for (int w = 0; w < (a.nhib + 63) / 64; ++w) nha += (int)s_wn[w];
        S dgh = (S)0;
        for (int b = 0; b < a.nhib; ++b) {
            const uint32_t mk = hib[b].mask;
            const uint32_t t = hh & mk;
            dgh += (t == 0u || t == mk) ? (S)hib[b].jz4 : -(S)hib[b].jz4;
        }
        if (a.hz)
            for (int i = a.n_lo; i < a.n_sites; ++i)
                dgh -= (S)a.hz[i] * (((hh >> (i - a.n_lo)) & 1u) ? (S)0.5 : (S)-0.5);
        for (uint32_t p = ps; p < L; p += sp) {
            const uint32_t g = g0 + p;
            const uint32_t l = lol[g];
            S acc[VPT];
#pragma unroll
            for (int j = 0; j < VPT; ++j) acc[j] = (S)0;
            S dg = dgh;
            if (a.hz)
                for (int i = 0; i < a.n_lo; ++i) dg -= (S)a.hz[i] * (((l >> i) & 1u) ? (S)0.5 : (S)-0.5);
            // bonds inside the low part: partners in LDS
            for (int b0 = 0; b0 < a.nlob; b0 += kBatchV) {
                uint32_t q[kBatchV];
                S cf[kBatchV];
                unsigned anti = 0u;
#pragma unroll
                for (int t = 0; t < kBatchV; ++t) {
                    q[t] = 0u;
                    cf[t] = (S)0;
                    const int b = b0 + t;
                    if (b < a.nlob) {
                        const uint32_t mk = lob[b].mask;
                        const uint32_t tt = l & mk;
                        const S jz = (S)lob[b].jz4;
                        if (tt == 0u || tt == mk) {
                            dg += jz;
                        } else {
                            dg -= jz;
                            anti |= 1u << t;
                            cf[t] = (S)lob[b].jxy2;
                        }
                        q[t] = tab[(uint64_t)lob[b].row * a.pitch + g];
                    }
                }
#pragma unroll
                for (int t = 0; t < kBatchV; ++t)
                    if (anti & (1u << t)) {
                        S x[VPT];
                        ld_piece<S, VPT>(blk + (size_t)q[t] * NV + sub * VPT, x);
#pragma unroll
                        for (int j = 0; j < VPT; ++j) acc[j] += cf[t] * x[j];
                    }
            }
            // bonds across the split: one state of a partner block
            for (int b0 = 0; b0 < a.nxb; b0 += kBatchV) {
                uint64_t src[kBatchV];
                S cf[kBatchV], val[kBatchV][VPT];
                unsigned anti = 0u;
#pragma unroll
                for (int t = 0; t < kBatchV; ++t) {
                    src[t] = 0;
                    cf[t] = (S)0;
                    const int b = b0 + t;
                    if (b < a.nxb) {
                        const uint32_t hbit = xb[b].hbit;
                        const uint64_t pb = hoff[hh ^ (1u << hbit)];
                        const uint32_t q = tab[(uint64_t)xb[b].row * a.pitch + g];
                        const uint32_t hb = (hh >> hbit) & 1u;
                        const uint32_t lb = (l >> xb[b].lbit) & 1u;
                        const S jz = (S)xb[b].jz4;
                        if (hb == lb) {
                            dg += jz;
                        } else {
                            dg -= jz;
                            anti |= 1u << t;
                            cf[t] = (S)xb[b].jxy2;
                            src[t] = pb + q;
                        }
                    }
                }
#pragma unroll
                for (int t = 0; t < kBatchV; ++t) {
                    if (anti & (1u << t)) ld_piece<S, VPT>(v + src[t] * NV + sub * VPT, val[t]);
                    else
#pragma unroll
                        for (int j = 0; j < VPT; ++j) val[t][j] = (S)0;
                }
#pragma unroll
                for (int t = 0; t < kBatchV; ++t)
                    if (anti & (1u << t))
#pragma unroll
                        for (int j = 0; j < VPT; ++j) acc[j] += cf[t] * val[t][j];
            }
            // bonds inside the high part: the same state of a partner
            // block, the block's flipping ones only
            for (int b0 = 0; b0 < nha; b0 += kBatchV) {
                S val[kBatchV][VPT];
#pragma unroll
                for (int t = 0; t < kBatchV; ++t) {
                    if (b0 + t < nha) ld_piece<S, VPT>(v + (s_hsrc[b0 + t] + p) * NV + sub * VPT, val[t]);
                    else
#pragma unroll
                        for (int j = 0; j < VPT; ++j) val[t][j] = (S)0;
                }
#pragma unroll
                for (int t = 0; t < kBatchV; ++t)
                    if (b0 + t < nha)
#pragma unroll
                        for (int j = 0; j < VPT; ++j) acc[j] += s_hcf[b0 + t] * val[t][j];
            }
            S me_v[VPT], hv[VPT], uu[VPT], out[VPT];
            ld_piece<S, VPT>(blk + (size_t)p * NV + sub * VPT, me_v);
#pragma unroll
            for (int j = 0; j < VPT; ++j) {
                hv[j] = acc[j] + dg * me_v[j];
                uu[j] = (S)0;
            }
            const size_t me = (size_t)(base + p) * NV + (size_t)sub * VPT;
            if (u) ld_piece<S, VPT>(u + me, uu);
            epilogue_r<S, VPT>(hv, uu, u != nullptr, a.coef_cplx, a.coef, out);
            st_piece<S, VPT>(w + me, out);
            if (rawp) st_piece<S, VPT>(rawp + me, hv);
            if (accp) {
#pragma unroll
                for (int j = 0; j < VPT; ++j) accp[me + j] += out[j];
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        s_last = (atomicAdd(&a.sched[1], 1u) == gridDim.x - 1) ? 1u : 0u;
        if (s_last) {
            a.sched[0] = 0u;
            a.sched[1] = 0u;
            __threadfence();
        }
    }
}

uint64_t binom_small(int n, int k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

// Largest block at split point nl: max over high popcounts k of
// C(nl, n_pop - k), k = 0..n_bits - nl.
uint64_t blk_max_len(int n_bits, int n_pop, int nl)
{
    uint64_t m = 0;
    for (int k = 0; k <= n_bits - nl; ++k) m = std::max(m, binom_small(nl, n_pop - k));
    return m;
}

// LDS of a block: at most all of a CU's 160 KB less the kernel's own shared
// words for a forced split point, a share that leaves room for
// blk_per_cu workgroups for the automatic one
constexpr size_t kBlkLdsMax = kCuLds - 256;
size_t blk_lds_share(int esize, bool f32) { return kCuLds / (size_t)blk_per_cu(esize, f32) - 256; }

// Split point, tables and bond lists for esize bytes per state.
int blk_tables(hphi_ham *h, int esize, bool f32)
{
    SpinBlk &B = h->blk;
    const Species &s = h->basis->sp[0];
    const int N = s.n_bits, np = s.n_pop, want = h->sched_cfg.spin_blk_lo;
    if (B.built && B.esize == esize && B.f32 == f32 && B.want == want) return HPHI_OK;
    const size_t budget = want > 0 ? kBlkLdsMax : blk_lds_share(esize, f32);
    int nl = 0;
    if (want > 0) {
        if (want > N || want > 24 || N - want > 24 || blk_max_len(N, np, want) * (uint64_t)esize > budget)
            return fail(HPHI_ERR_UNSUPPORTED, "spin_blk_lo %d: blocks of %d-byte states do not fit LDS", want, esize);
        nl = want;
    } else {
        for (int n = std::min(s.n_lo, 24); n >= 1 && N - n <= 24; --n)
            if (blk_max_len(N, np, n) * (uint64_t)esize <= budget) {
                nl = n;
                break;
            }
    }
    B.built = true;
    B.esize = esize;
    B.f32 = f32;
    B.want = want;
    B.ok = nl > 0;
    if (!B.ok) return HPHI_OK;
    if (B.sp && B.n_lo == nl) return HPHI_OK;   // same split point: tables kept
    auto sp = std::make_unique<Species>();
    HPHI_TRY(build_species(*sp, N, np, nl, false));
    const uint32_t nlo = 1u << nl;
    // bonds by where their ends fall
    std::vector<LoBondDev> lob;
    std::vector<XBondDev> xb;
    std::vector<HiBondDev> hib;
    std::vector<int> site_row(nl, -1);
    std::vector<uint32_t> low_masks, x_sites;
    for (const SpinBondDev &b : h->bonds) {
        const bool li = b.i < nl, lj = b.j < nl;
        if (li && lj) {
            LoBondDev d{};
            d.mask = (uint32_t)b.mask;
            d.row = (uint32_t)lob.size();
            d.jz4 = b.jz4;
            d.jxy2 = b.jxy2;
            lob.push_back(d);
            low_masks.push_back(d.mask);
        } else if (!li && !lj) {
            HiBondDev d{};
            d.mask = (uint32_t)(b.mask >> nl);
            d.jz4 = b.jz4;
            d.jxy2 = b.jxy2;
            hib.push_back(d);
        } else {
            XBondDev d{};
            d.lbit = (uint32_t)(li ? b.i : b.j);
            d.hbit = (uint32_t)((li ? b.j : b.i) - nl);
            if (site_row[d.lbit] < 0) {
                site_row[d.lbit] = (int)x_sites.size();
                x_sites.push_back(d.lbit);
            }
            d.jz4 = b.jz4;
            d.jxy2 = b.jxy2;
            xb.push_back(d);
        }
    }
    const uint32_t n_lob = (uint32_t)lob.size();
    for (XBondDev &d : xb) d.row = n_lob + (uint32_t)site_row[d.lbit];
    // bonds of one low site next to each other: a batch loads that site's
    // partner positions once
    std::stable_sort(xb.begin(), xb.end(), [](const XBondDev &x, const XBondDev &y) { return x.row < y.row; });
    // partner positions: low bond b at row b (rank of l ^ mask where the
    // bond is antiparallel, else 0); crossing site i at row n_lob + its
    // index (rank of l ^ bit i), over all low patterns by popcount group
    const size_t rows = low_masks.size() + x_sites.size();
    std::vector<uint16_t> tab(std::max<size_t>(rows, 1) * nlo, 0);
    for (uint32_t g = 0; g < nlo; ++g) {
        const uint32_t l = sp->lo_list[g];
        for (size_t r = 0; r < low_masks.size(); ++r) {
            const uint32_t mk = low_masks[r], t = l & mk;
            if (t != 0u && t != mk) tab[r * nlo + g] = (uint16_t)sp->lo_rank[l ^ mk];
        }
        for (size_t r = 0; r < x_sites.size(); ++r)
            tab[(low_masks.size() + r) * nlo + g] = (uint16_t)sp->lo_rank[l ^ (1u << x_sites[r])];
    }
    // blocks by popcount of h, ascending h within
    const int nh = N - nl;
    std::vector<uint32_t> list, len(nh + 1, 0), off(nh + 1, 0);
    for (int k = 0; k <= nh; ++k) {
        const int c = np - k;
        if (c < 0 || c > nl) continue;
        len[k] = (uint32_t)binom_small(nl, c);
        off[k] = sp->lo_list_off[c];
        for (uint32_t x = 0; x < (1u << nh); ++x)
            if (__builtin_popcount(x) == k) list.push_back(x);
    }
    if (hib.size() > (size_t)kMaxHiBonds || xb.size() > (size_t)kMaxHiBonds) {
        // the kernels list a block's flipping high bonds and its crossing
        // bonds' partner blocks in LDS
        B.ok = false;
        return HPHI_OK;
    }
    B.n_lob = (int)n_lob;
    B.n_xb = (int)xb.size();
    B.n_hib = (int)hib.size();
    if (lob.empty()) lob.push_back(LoBondDev{});
    if (xb.empty()) xb.push_back(XBondDev{});
    if (hib.empty()) hib.push_back(HiBondDev{});
    B.n_blocks = (uint32_t)list.size();
    B.max_len = (uint32_t)blk_max_len(N, np, nl);
    HPHI_TRY(upload(B.lob, lob.data(), sizeof(LoBondDev) * lob.size()));
    HPHI_TRY(upload(B.xb, xb.data(), sizeof(XBondDev) * xb.size()));
    HPHI_TRY(upload(B.hib, hib.data(), sizeof(HiBondDev) * hib.size()));
    HPHI_TRY(upload(B.tab, tab.data(), sizeof(uint16_t) * tab.size()));
    HPHI_TRY(upload(B.hi_list, list.data(), sizeof(uint32_t) * list.size()));
    HPHI_TRY(upload(B.cls_len, len.data(), sizeof(uint32_t) * len.size()));
    HPHI_TRY(upload(B.lo_off, off.data(), sizeof(uint32_t) * off.size()));
    B.sp = std::move(sp);
    B.n_lo = nl;
    return HPHI_OK;
}

template <typename S, int NV>
int launch_blk_t(hphi_ham *h, const MultArgs &m)
{
    const SpinBlk &B = h->blk;
    BlkKArgs a{};
    a.hi_list = B.hi_list.as<uint32_t>();
    a.n_blocks = B.n_blocks;
    a.hi_off = B.sp->d_hi_off.as<uint64_t>();
    a.lo_list = B.sp->d_lo_list.as<uint32_t>();
    a.cls_len = B.cls_len.as<uint32_t>();
    a.lo_off = B.lo_off.as<uint32_t>();
    a.lob = B.lob.as<LoBondDev>();
    a.xb = B.xb.as<XBondDev>();
    a.hib = B.hib.as<HiBondDev>();
    a.nlob = B.n_lob;
    a.nxb = B.n_xb;
    a.nhib = B.n_hib;
    a.tab = B.tab.as<uint16_t>();
    a.pitch = uint64_t(1) << B.n_lo;
    a.hz = h->has_field ? h->d_hz.as<double>() : nullptr;
    a.n_lo = B.n_lo;
    a.n_sites = h->basis->n_sites;
    a.sched = h->sched.as<unsigned>();
    a.v = m.v;
    a.w = m.w;
    a.u = m.u;
    a.acc_out = m.acc;
    a.coef = m.coef;
    a.raw_out = m.raw_out;
    a.coef_cplx = m.coef_cplx;
    constexpr int esize = NV * (int)sizeof(S);
    const size_t lds = (size_t)B.max_len * esize;
    const void *kern;
    if constexpr (NV == 1) kern = (const void *)k_spin_blk<S>;
    else kern = (const void *)k_spin_blk_v<S, NV>;
    HPHI_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int ncu = h->basis->ctx->n_cu > 0 ? h->basis->ctx->n_cu : 256;
    const uint32_t fit = (uint32_t)(kCuLds / (lds + 256));
    constexpr bool f32 = sizeof(S) == 4;
    const uint32_t per_cu = std::max(1u, std::min((uint32_t)blk_per_cu(esize, f32), fit));
    uint32_t grid = (uint32_t)ncu * per_cu;
    if (grid > B.n_blocks) grid = B.n_blocks;
    if constexpr (NV == 1)
        hipLaunchKernelGGL((k_spin_blk<S>), dim3(grid), dim3(blk_threads(esize, f32)), lds, m.stream, a);
    else
        hipLaunchKernelGGL((k_spin_blk_v<S, NV>), dim3(grid), dim3(blk_threads(esize, f32)), lds, m.stream, a);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace

int launch_spin_blk(hphi_ham *h, const MultArgs &m, int *done)
{
    *done = 0;
    const int nv = m.nvec * dtype_lanes(m.dtype);
    if (m.dots || m.cocg || (nv == 1 && m.raw_out)) return HPHI_OK;
    if (nv != 1 && nv != 2 && nv != 4 && nv != 8 && nv != 16 && nv != 32) return HPHI_OK;
    const bool f32 = dtype_is_f32(m.dtype);
    HPHI_TRY(blk_tables(h, nv * (f32 ? 4 : 8), f32));
    if (!h->blk.ok || h->blk.n_blocks == 0) return HPHI_OK;
    int rc = HPHI_OK;
    switch (nv) {
    case 1: rc = f32 ? launch_blk_t<float, 1>(h, m) : launch_blk_t<double, 1>(h, m); break;
    case 2: rc = f32 ? launch_blk_t<float, 2>(h, m) : launch_blk_t<double, 2>(h, m); break;
    case 4: rc = f32 ? launch_blk_t<float, 4>(h, m) : launch_blk_t<double, 4>(h, m); break;
    case 8: rc = f32 ? launch_blk_t<float, 8>(h, m) : launch_blk_t<double, 8>(h, m); break;
    case 16: rc = f32 ? launch_blk_t<float, 16>(h, m) : launch_blk_t<double, 16>(h, m); break;
    default: rc = f32 ? launch_blk_t<float, 32>(h, m) : launch_blk_t<double, 32>(h, m); break;
    }
    HPHI_TRY(rc);
    *done = 1;
    return HPHI_OK;
}

} // namespace hphi

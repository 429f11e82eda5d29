// Batched small-sector Lanczos: whole solves inside one launch.
//
// For sectors of up to a few hundred thousand states an H*v takes a few
// microseconds, so a solve driven by one kernel launch per step is bound by
// launch latency. Here a launch carries many independent requests (each its
// own spin Hamiltonian, sector, iteration count and seed) and runs the
// complete recurrence of each (the plain Lanczos of the HPhi update paper's
// introduction, without reorthogonalization):
//   q_0 = r (SplitMix64 uniform [-1/2, 1/2), the same stream as the
//   single-solve path), s_0 = 1/|q_0|;
//   w = s_k H q_k - beta_k s_{k-1} q_{k-1};  alpha_k = s_k <q_k, w>;
//   w -= alpha_k s_k q_k;  beta_{k+1} = |w|;  q_{k+1} = w, s_{k+1} = 1/beta_{k+1};
// either on one workgroup with the vector in LDS (many small requests:
// throughput) or on a team of workgroups that meet at a barrier of their own
// (few requests, or vectors too large for LDS: latency).
//
// Every reduction follows one order defined on the rows alone: each 64-row
// chunk is summed by one fixed cross-lane tree, the chunks of a 1024-row
// slice in order, then the slices in order. A request's numbers are
// therefore the same in either kernel, whatever the team width and whatever
// else shares the launch.
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
    int *done;          // [0] steps done, [1] breakdown flag (3: team barrier timed out)
    double *part;       // chunk partials (dim / 64, rounded up), then two buffers of slice sums
    unsigned *bar;      // team barrier arrivals (zero at launch)
    int team_base;      // first arrival ticket of the request's team
    int team_w;         // members in the team
    int team_rows;      // rows per member, a multiple of the slice
};

constexpr int kBatchLdsTab = 8192;   // uint32 entries of staged tables
constexpr int kChunk = 64;           // rows per chunk partial (one wave)
constexpr int kSlice = 16;           // chunks per slice
constexpr unsigned kTeamSpin = 1u << 25;   // polls before a barrier gives up (seconds)
constexpr int kTeamMax = 32;               // workgroups per request at most

__host__ __device__ __forceinline__ int64_t n_chunks(int64_t dim) { return (dim + kChunk - 1) / kChunk; }

// One DPP move of a double (both halves); lanes without a source read 0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROW_MASK, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROW_MASK, 0xF, false);
    return __hiloint2double(hi, lo);
}

// The wave's 64 row contributions -> part[c], by one fixed tree: shifts by
// 1, 2, 4 and 8 lanes within each 16-lane row (lane 15 of a row then holds
// the row's sum), lane 15 of rows 0 and 2 added into rows 1 and 3, then
// lane 31 into rows 2 and 3; lane 63 holds the total and stores it. Every
// lane of the wave must be active.
__device__ __forceinline__ void chunk_store(double v, double *part, int64_t c)
{
    v += dpp_f64<0x111, 0xF>(v);   // row_shr:1
    v += dpp_f64<0x112, 0xF>(v);   // row_shr:2
    v += dpp_f64<0x114, 0xF>(v);   // row_shr:4
    v += dpp_f64<0x118, 0xF>(v);   // row_shr:8
    v += dpp_f64<0x142, 0xA>(v);   // row_bcast:15
    v += dpp_f64<0x143, 0xC>(v);   // row_bcast:31
    if ((threadIdx.x & (kWave - 1)) == kWave - 1) part[c] = v;
}

// Slice s of the chunk partials, summed in chunk order (all loads in flight
// first; a chunk past the end adds exactly +0).
__device__ __forceinline__ double slice_sum(const double *part, int64_t s, int64_t nch)
{
    double v[kSlice];
#pragma unroll
    for (int j = 0; j < kSlice; ++j) {
        const int64_t c = s * kSlice + j;
        v[j] = c < nch ? part[c] : 0.0;
    }
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < kSlice; ++j) t += v[j];
    return t;
}

// Sum of the ns slice values in order; one whole wave calls it and every
// lane returns the same value. With FROM_CHUNKS the slice values are summed
// from the chunk partials here, otherwise they are read from `v`.
template <bool FROM_CHUNKS>
__device__ __forceinline__ double ordered_total(const double *v, int64_t nch)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t ns = (nch + kSlice - 1) / kSlice;
    double tot = 0.0;
    for (int64_t s0 = 0; s0 < ns; s0 += kWave) {
        const int64_t s = s0 + lane;
        double S = 0.0;
        if (s < ns) S = FROM_CHUNKS ? slice_sum(v, s, nch) : v[s];
        const int cnt = (int)min((int64_t)kWave, ns - s0);
        for (int j = 0; j < cnt; ++j) tot += __shfl(S, j, kWave);
    }
    return tot;
}

// Workgroup-wide ordered total of the chunk partials just stored by this
// workgroup (the one-workgroup kernel).
__device__ __forceinline__ double block_total(const double *part, int64_t nch, double *bcast)
{
    __syncthreads();
    if (threadIdx.x < kWave) {
        const double t = ordered_total<true>(part, nch);
        if (threadIdx.x == 0) *bcast = t;
    }
    __syncthreads();
    const double r = *bcast;
    __syncthreads();
    return r;
}

// Bond sums of one state: the off-diagonal gathers and the diagonal. With
// BATCH (vectors in global memory) eight bonds go per batch, their targets
// first, then all eight loads in flight, then the sums in bond order, a bond
// without a flip adding exactly +0; without (vector in LDS) only the flips
// load. Both add the same terms in the same order.
template <bool BATCH, typename RankFn>
__device__ __forceinline__ void spin_row(const BatchItemDev &it, const CSpinBond *bc, const CDouble *hzc, uint32_t x,
                                         int64_t r, const double *qc, RankFn rank, double &hv, double &diag)
{
    hv = 0.0;
    diag = 0.0;
    if (!BATCH) {
        for (int b = 0; b < it.nb; ++b) {
            const uint32_t m = (uint32_t)bc[b].mask, t = x & m;
            if (t == 0u || t == m) {
                diag += bc[b].jz4;
            } else {
                diag -= bc[b].jz4;
                hv += bc[b].jxy2 * qc[rank(x ^ m)];
            }
        }
    }
    for (int b0 = 0; BATCH && b0 < it.nb; b0 += 8) {
        uint32_t idx[8];
        double cf[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            idx[k] = (uint32_t)r;
            cf[k] = 0.0;
            const int b = b0 + k;
            if (b < it.nb) {
                const uint32_t m = (uint32_t)bc[b].mask, t = x & m;
                if (t == 0u || t == m) {
                    diag += bc[b].jz4;
                } else {
                    diag -= bc[b].jz4;
                    idx[k] = rank(x ^ m);
                    cf[k] = bc[b].jxy2;
                }
            }
        }
        double nv[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) nv[k] = qc[idx[k]];
#pragma unroll
        for (int k = 0; k < 8; ++k) hv += cf[k] * nv[k];
    }
    if (it.hz)
        for (int i = 0; i < it.n_sites; ++i) diag -= hzc[i] * (((x >> i) & 1u) ? 0.5 : -0.5);
}

// LDS-resident variant for sectors whose vector fits next to the rank
// tables in LDS: q_k and the chunk partials live in LDS (the H*v gathers
// read q_k there), q_{k-1} and w in global memory. The update step moves q_k to the q_{k-1} buffer
// and writes q_{k+1} into LDS row by row (each thread touches only its own
// rows), so a step is one gather pass from LDS plus four streaming passes.
constexpr int kBatchLdsThreads = 1024;

__global__ __launch_bounds__(kBatchLdsThreads) void k_lanczos_batch_lds(const BatchItemDev *items)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ double bcast;
    const BatchItemDev it = items[blockIdx.x];
    // uniform tables through the scalar cache (the item is read from memory,
    // so without the cast every lane would load them with vector loads)
    const CSpinBond *bc = (const CSpinBond *)(it.bonds);
    const CDouble *hzc = (const CDouble *)(it.hz);
    const int64_t dim = it.dim, nch = n_chunks(dim);
    double *Q = reinterpret_cast<double *>(smem_raw);
    double *part = Q + dim;   // chunk partials, in LDS here
    uint32_t *lo = reinterpret_cast<uint32_t *>(part + nch);
    const uint32_t nl = 1u << it.n_lo, nh = 1u << it.n_hi;
    uint32_t *hi = lo + nl;
    for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) lo[i] = it.lo_rank[i];
    for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) hi[i] = it.hi_off[i];
    const uint32_t lomask = nl - 1u;
    const int n_lo = it.n_lo;
    auto rank = [&](uint32_t y) -> uint32_t { return hi[y >> n_lo] + lo[y & lomask]; };
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wrow = threadIdx.x & ~(kWave - 1);
    double *P = it.q, *Wv = it.q + dim;
    for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
        const int64_t r = b0 + lane;
        double c = 0.0;
        if (r < dim) {
            const double x = u53(splitmix64_at(it.seed, (uint64_t)r)) - 0.5;
            Q[r] = x;
            c = x * x;
        }
        chunk_store(c, part, b0 / kChunk);
    }
    const double n0 = block_total(part, nch, &bcast);
    double s_cur = 1.0 / sqrt(n0), s_prev = 0.0, b_cur = 0.0;
    int k = 0, brk = 0;
    for (; k < it.iters; ++k) {
        const double c1 = s_cur, c2 = -b_cur * s_prev;
        for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
            const int64_t r = b0 + lane;
            double c = 0.0;
            if (r < dim) {
                double hv, diag;
                spin_row<false>(it, bc, hzc, it.states[r], r, Q, rank, hv, diag);
                const double qr = Q[r];
                double o = c1 * (hv + diag * qr);
                if (k > 0) o += c2 * P[r];
                Wv[r] = o;
                c = qr * o;
            }
            chunk_store(c, part, b0 / kChunk);
        }
        const double al = s_cur * block_total(part, nch, &bcast);
        const double f = al * s_cur;
        for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
            const int64_t r = b0 + lane;
            double c = 0.0;
            if (r < dim) {
                const double qr = Q[r];
                const double x = Wv[r] - f * qr;
                P[r] = qr;
                Q[r] = x;
                c = x * x;
            }
            chunk_store(c, part, b0 / kChunk);
        }
        const double bn = sqrt(block_total(part, nch, &bcast));
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

// Team variant: request b runs on team_w workgroups, member m owning rows
// [m * team_rows, (m + 1) * team_rows) of every vector (whole slices). Per
// step the members meet twice, after the <q_k, w> slice sums and after the
// |w|^2 slice sums, and every member adds the slice sums in order, so all
// of them hold the same alpha and beta bits and take the same branch.
// Members take their place from an arrival ticket: the arrived workgroups
// form complete teams except at most the last one, and complete teams finish
// on their own, so the launch progresses even while other work holds part of
// the GPU. A barrier that still waits after kTeamSpin polls sets the
// request's flag to 3 and its members leave, so every wave ends.
__device__ __forceinline__ bool team_sync(unsigned *bar, unsigned target, int tw, int *s_fail)
{
    // the workgroup barrier orders every wave's stores before thread 0's
    // agent-scope release; thread 0's acquire fence after the polls (relaxed,
    // so that waiting does not invalidate the XCD's L2 once per poll) orders
    // the other members' stores before every wave's loads
    __syncthreads();
    if (tw > 1 && threadIdx.x == 0) {
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned polls = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(4);
            if (++polls >= kTeamSpin) {
                *s_fail = 1;
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return *s_fail != 0;
}

// 1024 threads: one row per thread for members of one slice, so all of a
// member's gathers are in flight at once.
constexpr int kTeamThreads = 1024;

__global__ __launch_bounds__(kTeamThreads) void k_lanczos_team(const BatchItemDev *items, int n, unsigned *ticket)
{
    __shared__ double bcast;
    __shared__ unsigned s_ticket;
    __shared__ int s_fail;
    __shared__ uint32_t s_tab[kBatchLdsTab];
    if (threadIdx.x == 0) {
        s_ticket = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_fail = 0;
    }
    __syncthreads();
    const int tk = (int)s_ticket;
    // request whose ticket range holds tk (items sorted by team_base)
    int lo_i = 0, hi_i = n - 1;
    while (lo_i < hi_i) {
        const int mid = (lo_i + hi_i + 1) >> 1;
        if (items[mid].team_base <= tk) lo_i = mid;
        else hi_i = mid - 1;
    }
    const BatchItemDev it = items[lo_i];
    const int mem = tk - it.team_base, tw = it.team_w;
    const CSpinBond *bc = (const CSpinBond *)(it.bonds);
    const CDouble *hzc = (const CDouble *)(it.hz);
    const int64_t dim = it.dim, nch = n_chunks(dim);
    const int64_t rbeg = (int64_t)mem * it.team_rows, rend = min(dim, rbeg + it.team_rows);
    const int64_t s_beg = rbeg / (kChunk * kSlice);
    const int64_t s_end = (rend + kChunk * kSlice - 1) / (kChunk * kSlice);
    // slice sums, two buffers used by turns: a member may write the next
    // barrier's sums while a slower one still reads the last barrier's
    const int64_t ns = (nch + kSlice - 1) / kSlice;
    int turn = 0;
    const uint32_t lomask = (1u << it.n_lo) - 1u;
    const uint32_t nl = 1u << it.n_lo, nh = 1u << it.n_hi;
    const uint32_t *lo = it.lo_rank, *hi = it.hi_off;
    if (nl + nh <= (uint32_t)kBatchLdsTab) {
        for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) s_tab[i] = it.lo_rank[i];
        for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) s_tab[nl + i] = it.hi_off[i];
        lo = s_tab;
        hi = s_tab + nl;
    }
    const int n_lo = it.n_lo;
    auto rank = [&](uint32_t y) -> uint32_t { return hi[y >> n_lo] + lo[y & lomask]; };
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wrow = rbeg + (threadIdx.x & ~(kWave - 1));
    unsigned arrivals = 0;
    // this member's slice sums -> ssum, barrier, then the ordered total of
    // all slice sums (identical in every member)
    auto team_total = [&](double &out) -> bool {
        double *ssum = it.part + nch + (turn ? ns : 0);
        turn ^= 1;
        __syncthreads();
        if (threadIdx.x < kWave)
            for (int64_t s = s_beg + lane; s < s_end; s += kWave) ssum[s] = slice_sum(it.part, s, nch);
        arrivals += (unsigned)tw;
        if (team_sync(it.bar, arrivals, tw, &s_fail)) return false;
        if (threadIdx.x < kWave) {
            const double t = ordered_total<false>(ssum, nch);
            if (threadIdx.x == 0) bcast = t;
        }
        __syncthreads();
        out = bcast;
        __syncthreads();
        return true;
    };
    double *q[3] = {it.q, it.q + dim, it.q + 2 * dim};
    int k = 0, brk = 0;
    double n0;
    for (int64_t b0 = wrow; b0 < rend; b0 += blockDim.x) {
        const int64_t r = b0 + lane;
        double c = 0.0;
        if (r < rend) {
            const double x = u53(splitmix64_at(it.seed, (uint64_t)r)) - 0.5;
            q[0][r] = x;
            c = x * x;
        }
        chunk_store(c, it.part, b0 / kChunk);
    }
    if (!team_total(n0)) goto timed_out;
    {
        double s_cur = 1.0 / sqrt(n0), s_prev = 0.0, b_cur = 0.0;
        int cur = 0, prev = 2, wb = 1;
        for (; k < it.iters; ++k) {
            const double c1 = s_cur, c2 = -b_cur * s_prev;
            const double *qc = q[cur], *qp = q[prev];
            double *w = q[wb];
            for (int64_t b0 = wrow; b0 < rend; b0 += blockDim.x) {
                const int64_t r = b0 + lane;
                double c = 0.0;
                if (r < rend) {
                    double hv, diag;
                    spin_row<true>(it, bc, hzc, it.states[r], r, qc, rank, hv, diag);
                    const double qr = qc[r];
                    double o = c1 * (hv + diag * qr);
                    if (k > 0) o += c2 * qp[r];
                    w[r] = o;
                    c = qr * o;
                }
                chunk_store(c, it.part, b0 / kChunk);
            }
            double pa;
            if (!team_total(pa)) goto timed_out;
            const double al = s_cur * pa;
            const double f = al * s_cur;
            for (int64_t b0 = wrow; b0 < rend; b0 += blockDim.x) {
                const int64_t r = b0 + lane;
                double c = 0.0;
                if (r < rend) {
                    const double x = w[r] - f * qc[r];
                    w[r] = x;
                    c = x * x;
                }
                chunk_store(c, it.part, b0 / kChunk);
            }
            double pb;
            if (!team_total(pb)) goto timed_out;
            const double bn = sqrt(pb);
            if (mem == 0 && threadIdx.x == 0) {
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
    }
    if (mem == 0 && threadIdx.x == 0) {
        it.done[0] = k;
        atomicMax(it.done + 1, brk);
        it.beta[0] = 0.0;
    }
    return;
timed_out:
    if (threadIdx.x == 0) {
        if (mem == 0) it.done[0] = k;
        atomicMax(it.done + 1, 3);
    }
}

size_t batch_lds_bytes(int64_t dim, int n_lo, int n_hi)
{
    return sizeof(double) * (size_t)(dim + n_chunks(dim)) +
           sizeof(uint32_t) * ((size_t(1) << n_lo) + (size_t(1) << n_hi));
}

size_t batch_part_doubles(int64_t dim)
{
    const int64_t nch = n_chunks(dim), ns = (nch + kSlice - 1) / kSlice;
    return (size_t)(nch + 2 * ns);
}

void batch_team_shape(int64_t dim, int *w, int *rows)
{
    const int64_t sl = (int64_t)kChunk * kSlice;
    const int64_t per = (dim + kTeamMax - 1) / kTeamMax;
    const int64_t r = std::max<int64_t>(sl, (per + sl - 1) / sl * sl);
    *rows = (int)r;
    *w = (int)std::max<int64_t>(1, (dim + r - 1) / r);
}

int launch_lanczos_team(const void *items_dev, int n, int grid, unsigned *ticket, hipStream_t st)
{
    hipLaunchKernelGGL(k_lanczos_team, dim3(grid), dim3(kTeamThreads), 0, st, (const BatchItemDev *)items_dev, n,
                       ticket);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_lanczos_batch(const void *items_dev, int n, hipStream_t st, size_t lds_bytes)
{
    HPHI_HIP(hipFuncSetAttribute((const void *)k_lanczos_batch_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_bytes));
    hipLaunchKernelGGL(k_lanczos_batch_lds, dim3(n), dim3(kBatchLdsThreads), lds_bytes, st,
                       (const BatchItemDev *)items_dev);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// ------------------------------------------------------ batched COCG --
// One (request, part of b) shifted-COCG sequence per 1024-thread workgroup
// (the scalar recurrences of kern_methods.hip, restated per workgroup):
// the request's rank tables in LDS, p, r and H p in global memory, every
// reduction in the row order of the batched Lanczos (64-row chunks by one
// DPP tree, then chunks in order), the per-shift scalars in global memory
// updated by one thread each. The part's norm decides, as in hphi_sqw,
// whether the sequence runs at all.
struct CocgItemDev {
    const uint32_t *states;
    int64_t dim;
    const SpinBondDev *bonds;
    int nb;
    int n_lo, n_hi;
    const uint32_t *lo_rank, *hi_off;
    const double *hz;
    int n_sites;
    const double *b;       // complex b, interleaved (re, im)
    int part;              // 0: Re b, 1: Im b
    double *r, *p, *h;     // complex, 2 dim doubles each
    double *chunks;        // 5 n_chunks(dim) doubles
    ShiftDev *sh;          // nsh shifts (sigma set)
    int nsh;
    double zs_re, zs_im;
    double tol;
    int max_iter;
    double *out;           // [0] iterations, [1] converged, [2] breakdown, [3] |part|^2, [4] |b|^2, [5] skipped
};

size_t cocg_item_size() { return sizeof(CocgItemDev); }

__global__ __launch_bounds__(kBatchLdsThreads) void k_cocg_batch(const CocgItemDev *items)
{
    extern __shared__ unsigned char smem_raw[];
    __shared__ double bcast;
    __shared__ double s_max[kBatchLdsThreads / kWave];
    const CocgItemDev it = items[blockIdx.x];
    const CSpinBond *bc = (const CSpinBond *)(it.bonds);
    const CDouble *hzc = (const CDouble *)(it.hz);
    const int64_t dim = it.dim, nch = n_chunks(dim);
    uint32_t *lo = reinterpret_cast<uint32_t *>(smem_raw);
    const uint32_t nl = 1u << it.n_lo, nh = 1u << it.n_hi;
    uint32_t *hi = lo + nl;
    for (uint32_t i = threadIdx.x; i < nl; i += blockDim.x) lo[i] = it.lo_rank[i];
    for (uint32_t i = threadIdx.x; i < nh; i += blockDim.x) hi[i] = it.hi_off[i];
    const uint32_t lomask = nl - 1u;
    const int n_lo = it.n_lo;
    auto rank = [&](uint32_t y) -> uint32_t { return hi[y >> n_lo] + lo[y & lomask]; };
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wrow = threadIdx.x & ~(kWave - 1);
    double *C0 = it.chunks, *C1 = C0 + nch, *C2 = C1 + nch, *C3 = C2 + nch, *C4 = C3 + nch;
    double2 *R = reinterpret_cast<double2 *>(it.r);
    double2 *P = reinterpret_cast<double2 *>(it.p);
    double2 *Hp = reinterpret_cast<double2 *>(it.h);
    const double2 *B = reinterpret_cast<const double2 *>(it.b);
    // norms of the two parts of b
    for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
        const int64_t r = b0 + lane;
        double a0 = 0.0, a1 = 0.0;
        if (r < dim) {
            const double2 bb = B[r];
            a0 = bb.x * bb.x;
            a1 = bb.y * bb.y;
        }
        chunk_store(a0, C0, b0 / kChunk);
        chunk_store(a1, C1, b0 / kChunk);
    }
    const double bn2_0 = block_total(C0, nch, &bcast);
    const double bn2_1 = block_total(C1, nch, &bcast);
    const double bn2 = it.part ? bn2_1 : bn2_0;
    const double bnorm = sqrt(bn2_0 + bn2_1);
    const double bsum = sqrt(bn2_0) + sqrt(bn2_1);
    const double tol_part = bsum > 0.0 ? it.tol * bnorm / bsum : it.tol;
    if (bn2 == 0.0 || sqrt(bn2) <= it.tol * bnorm) {
        // nothing to iterate (x_part = 0); the caller counts the part's norm
        for (int j = threadIdx.x; j < it.nsh; j += blockDim.x) {
            it.sh[j].X = {0.0, 0.0};
            it.sh[j].res = 0.0;
        }
        if (threadIdx.x == 0) {
            it.out[0] = 0.0; it.out[1] = 1.0; it.out[2] = 0.0;
            it.out[3] = bn2; it.out[4] = bn2_0 + bn2_1; it.out[5] = 1.0;
        }
        return;
    }
    // r = p = the part, as a complex vector
    for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
        const double2 bb = B[r];
        const double v = it.part ? bb.y : bb.x;
        R[r] = make_double2(v, 0.0);
        P[r] = make_double2(v, 0.0);
    }
    for (int j = threadIdx.x; j < it.nsh; j += blockDim.x) {
        ShiftDev s = it.sh[j];
        s.pi = {1.0, 0.0};
        s.pi_prev = {1.0, 0.0};
        s.X = {0.0, 0.0};
        s.P = {bn2, 0.0};
        s.res = 1.0;
        s.conv = 0;
        it.sh[j] = s;
    }
    const cd zs = {it.zs_re, it.zs_im};
    cd rho = {bn2, 0.0}, al = {1.0, 0.0}, be = {0.0, 0.0}, alp, bep;
    const double bn = sqrt(bn2);
    int iter = 0, conv = 0, brk = 0;
    double max_res = 1.0;
    __syncthreads();
    while (iter < it.max_iter) {
        // h = H p and the rows' terms of mu = p^T (z_s p - h)
        for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
            const int64_t r = b0 + lane;
            double m0 = 0.0, m1 = 0.0;
            if (r < dim) {
                const uint32_t x = it.states[r];
                double hr = 0.0, hi_ = 0.0, diag = 0.0;
                for (int b = 0; b < it.nb; b += 8) {
                    uint32_t idx[8];
                    double cf[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        idx[k] = (uint32_t)r;
                        cf[k] = 0.0;
                        if (b + k < it.nb) {
                            const uint32_t m = (uint32_t)bc[b + k].mask, t = x & m;
                            if (t == 0u || t == m) {
                                diag += bc[b + k].jz4;
                            } else {
                                diag -= bc[b + k].jz4;
                                idx[k] = rank(x ^ m);
                                cf[k] = bc[b + k].jxy2;
                            }
                        }
                    }
                    double2 nv[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) nv[k] = P[idx[k]];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        hr += cf[k] * nv[k].x;
                        hi_ += cf[k] * nv[k].y;
                    }
                }
                if (it.hz)
                    for (int i = 0; i < it.n_sites; ++i) diag -= hzc[i] * (((x >> i) & 1u) ? 0.5 : -0.5);
                const double2 pp = P[r];
                hr += diag * pp.x;
                hi_ += diag * pp.y;
                Hp[r] = make_double2(hr, hi_);
                const cd t = cmul(cd{pp.x, pp.y}, csub(cmul(zs, cd{pp.x, pp.y}), cd{hr, hi_}));
                m0 = t.re;
                m1 = t.im;
            }
            chunk_store(m0, C0, b0 / kChunk);
            chunk_store(m1, C1, b0 / kChunk);
        }
        const cd mu = {block_total(C0, nch, &bcast), block_total(C1, nch, &bcast)};
        alp = al;
        bep = be;
        if (cabs2(mu) == 0.0) {
            brk = 1;
            break;
        }
        al = cdiv(rho, mu);
        // r -= alpha (z_s p - h); rho' = r^T r, |r|^2, b^H r (b = the part)
        for (int64_t b0 = wrow; b0 < dim; b0 += blockDim.x) {
            const int64_t r = b0 + lane;
            double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
            if (r < dim) {
                const double2 pp = P[r], hh = Hp[r], rr = R[r], bb = B[r];
                const double bv = it.part ? bb.y : bb.x;
                const cd ap = csub(cmul(zs, cd{pp.x, pp.y}), cd{hh.x, hh.y});
                const cd rv = csub(cd{rr.x, rr.y}, cmul(al, ap));
                R[r] = make_double2(rv.re, rv.im);
                a[0] = rv.re * rv.re - rv.im * rv.im;
                a[1] = 2 * rv.re * rv.im;
                a[2] = rv.re * rv.re + rv.im * rv.im;
                a[3] = bv * rv.re;
                a[4] = bv * rv.im;
            }
            chunk_store(a[0], C0, b0 / kChunk);
            chunk_store(a[1], C1, b0 / kChunk);
            chunk_store(a[2], C2, b0 / kChunk);
            chunk_store(a[3], C3, b0 / kChunk);
            chunk_store(a[4], C4, b0 / kChunk);
        }
        const cd rho1 = {block_total(C0, nch, &bcast), block_total(C1, nch, &bcast)};
        const double rn = sqrt(block_total(C2, nch, &bcast));
        const cd bhr = {block_total(C3, nch, &bcast), block_total(C4, nch, &bcast)};
        if (cabs2(rho) == 0.0) {
            brk = 1;
            be = {0.0, 0.0};
        } else {
            be = cdiv(rho1, rho);
        }
        rho = rho1;
        ++iter;
        // per-shift recurrences (one thread per shift), then the largest
        // residual of the unconverged shifts
        const cd ratio = cabs2(alp) > 0.0 ? cdiv(cmul(al, bep), alp) : cd{0.0, 0.0};
        double mx = 0.0;
        for (int j = threadIdx.x; j < it.nsh; j += blockDim.x) {
            ShiftDev s = it.sh[j];
            if (!s.conv) {
                const cd one = {1.0, 0.0};
                const cd f = cadd(cadd(one, ratio), cmul(al, s.sigma));
                const cd pin = csub(cmul(f, s.pi), cmul(ratio, s.pi_prev));
                const cd q = cdiv(s.pi, pin);
                const cd als = cmul(q, al);
                const cd bes = cmul(cmul(q, q), be);
                s.X = cadd(s.X, cmul(als, s.P));
                s.P = cadd(cdiv(bhr, pin), cmul(bes, s.P));
                s.pi_prev = s.pi;
                s.pi = pin;
                s.res = rn / sqrt(cabs2(pin)) / bn;
                if (s.res < tol_part) s.conv = 1;
                it.sh[j] = s;
            }
            mx = fmax(mx, s.conv ? 0.0 : s.res);
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
        if (lane == 0) s_max[threadIdx.x >> 6] = mx;
        // p = r + beta p
        for (int64_t r = threadIdx.x; r < dim; r += blockDim.x) {
            const double2 rr = R[r], pp = P[r];
            const cd t = cmul(be, cd{pp.x, pp.y});
            P[r] = make_double2(rr.x + t.re, rr.y + t.im);
        }
        __syncthreads();
        max_res = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) max_res = fmax(max_res, s_max[w]);
        __syncthreads();
        if (iter % 8 == 0 || iter == it.max_iter) {
            if (max_res < tol_part) {
                conv = 1;
                break;
            }
            if (brk) break;
        }
    }
    if (threadIdx.x == 0) {
        it.out[0] = iter;
        it.out[1] = conv;
        it.out[2] = brk;
        it.out[3] = bn2;
        it.out[4] = bn2_0 + bn2_1;
        it.out[5] = 0.0;
    }
}

int fill_cocg_item(hphi_ham *h, const void *b, int part, double *r, double *p, double *hv, double *chunks,
                   void *sh, int nsh, double zs_re, double zs_im, double tol, int max_iter, double *out, void *dst)
{
    const hphi_basis *bs = h->basis;
    const Species &s = bs->sp[0];
    if (h->kind != 0 || !s.materialized() || s.state_bytes != 4 || !s.d_hi_off32.p)
        return fail(HPHI_ERR_UNSUPPORTED, "batched S(q, w) takes spin Hamiltonians with a stored basis");
    if ((1u << s.n_lo) + (1u << s.n_hi) > (unsigned)kBatchLdsTab)
        return fail(HPHI_ERR_UNSUPPORTED, "batched S(q, w): rank tables of %d sites exceed LDS", bs->n_sites);
    CocgItemDev d{};
    d.states = s.d_states.as<uint32_t>();
    d.dim = s.dim;
    d.bonds = h->d_bonds.as<SpinBondDev>();
    d.nb = h->n_bonds;
    d.n_lo = s.n_lo;
    d.n_hi = s.n_hi;
    d.lo_rank = s.d_lo_rank.as<uint32_t>();
    d.hi_off = s.d_hi_off32.as<uint32_t>();
    d.hz = h->has_field ? h->d_hz.as<double>() : nullptr;
    d.n_sites = bs->n_sites;
    d.b = static_cast<const double *>(b);
    d.part = part;
    d.r = r;
    d.p = p;
    d.h = hv;
    d.chunks = chunks;
    d.sh = static_cast<ShiftDev *>(sh);
    d.nsh = nsh;
    d.zs_re = zs_re;
    d.zs_im = zs_im;
    d.tol = tol;
    d.max_iter = max_iter;
    d.out = out;
    *static_cast<CocgItemDev *>(dst) = d;
    return HPHI_OK;
}

int launch_cocg_batch(const void *items_dev, int n, hipStream_t st)
{
    const size_t lds = sizeof(uint32_t) * kBatchLdsTab;
    HPHI_HIP(hipFuncSetAttribute((const void *)k_cocg_batch, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_cocg_batch, dim3(n), dim3(kBatchLdsThreads), lds, st, (const CocgItemDev *)items_dev);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int64_t cocg_chunks(int64_t dim) { return n_chunks(dim); }

size_t batch_item_size() { return sizeof(BatchItemDev); }

int fill_batch_item(hphi_ham *h, int iters, uint64_t seed, double *q, double *alpha, double *beta, int *done,
                    double *part, unsigned *bar, int team_base, void *out)
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
    d.part = part;
    d.bar = bar;
    d.team_base = team_base;
    batch_team_shape(s.dim, &d.team_w, &d.team_rows);
    *static_cast<BatchItemDev *>(out) = d;
    return HPHI_OK;
}

} // namespace hphi

// Internal declarations of the HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "../../include/hphi_mi355.h"
#include "use_guard.h"

namespace hphi {

// Record a failure (thread-local message) and return `code`.
int fail(int code, const char *fmt, ...);
const char *last_error();

#define HPHI_HIP(expr)                                                              \
    do {                                                                            \
        hipError_t e_ = (expr);                                                     \
        if (e_ != hipSuccess)                                                       \
            return ::hphi::fail(HPHI_ERR_DEVICE, "%s failed: %s (%s:%d)", #expr,   \
                                hipGetErrorString(e_), __FILE__, __LINE__);         \
    } while (0)

#define HPHI_TRY(expr)                \
    do {                              \
        int rc_ = (expr);             \
        if (rc_ != HPHI_OK) return rc_; \
    } while (0)

// Owning device allocation.
struct DevMem {
    void *p = nullptr;
    size_t bytes = 0;
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { reset(); }
    int alloc(size_t n);
    void reset();
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Both complete before returning (ordered before any later launch on any stream).
int upload(DevMem &m, const void *host, size_t bytes);
int zero_now(void *p, size_t bytes);

// Makes `dev` current for the scope, restores the previous device after.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};


// One species' sector: n_bits-bit patterns with n_pop set bits, ascending,
// ranked by the split two-level table idx = hi_off[x >> n_lo] + lo_rank[x & mask].
struct Species {
    int n_bits = 0, n_pop = 0, n_lo = 0, n_hi = 0;
    int64_t dim = 0;
    std::vector<uint32_t> lo_rank;      // 2^n_lo
    std::vector<uint64_t> hi_off;       // 2^n_hi + 1
    std::vector<uint32_t> lo_list;      // lo patterns grouped by popcount
    std::vector<uint32_t> lo_list_off;  // n_lo + 2 group offsets
    DevMem d_lo_rank, d_hi_off, d_hi_off32, d_lo_list, d_lo_list_off;
    DevMem d_states;                    // materialized states (uint32 or uint64) or empty
    int state_bytes = 0;
    bool materialized() const { return d_states.p != nullptr; }
    uint64_t state_at(int64_t r) const;  // host unrank via the tables
    int64_t rank_of(uint64_t x) const;   // host rank, -1 if outside
};

// Host tables only (no device memory touched).
int build_species_tables(Species &s, int n_bits, int n_pop, int n_lo_override);
int build_species(Species &s, int n_bits, int n_pop, int n_lo_override, bool materialize);

} // namespace hphi

struct hphi_ctx {
    int device = 0;
    int n_cu = 0;
    size_t lds_per_block = 0;
};

// Spin-S sector tables (basis kind 3): digits of b bits per site, split
// two-level rank idx = hi_off[x >> lo_bits] + lo_rank[x & (2^lo_bits - 1)].
struct SpinSTables {
    int two_s = 0, bits = 0, lo_bits = 0, hi_bits = 0, msum = 0;
    std::vector<uint32_t> lo_rank;    // 2^lo_bits (invalid patterns: ~0)
    std::vector<uint64_t> hi_off;     // 2^hi_bits + 1
    std::vector<uint64_t> states;     // host copy, ascending
    hphi::DevMem d_lo_rank, d_hi_off32, d_states;
    int64_t rank_of(uint64_t x) const;
};

struct hphi_basis {
    hphi_ctx *ctx = nullptr;
    int kind = 0;  // 0 = spin, 1 = Hubbard, 2 = spin on the full 2^N space (SpinGC), 3 = spin-S
    int n_sites = 0;
    int64_t dim = 0;
    hphi::Species sp[2];
    SpinSTables ss;
};

namespace hphi {

// Spin bond as the kernels read it.
struct SpinBondDev {
    uint64_t mask;   // (1 << i) | (1 << j)
    double jz4;      // jz / 4
    double jxy2;     // jxy / 2
    int32_t i, j;
    int32_t pad0, pad1;
};

// Two-body term of one site pair as the kernels read it.
struct HubPairDev {
    uint32_t mask;      // (1 << i) | (1 << j)
    uint32_t between;   // sites strictly between i and j
    int32_t i, j;
    double v, jh, jx, jp;
};
constexpr int kMaxPairTerms = 1024;
struct PairNbrDev {
    int32_t other, pad;
    double v;
};

// Split spin H*v: a bond with both ends in the high half of the sites, in
// high-half coordinates.
struct HiBondDev {
    uint32_t mask, pad;
    double jz4, jxy2;
};
constexpr int kMaxHiBonds = 128;
// Block-staged spin H*v (implicit basis): bonds by where their ends fall
// against a split point n_lo of the sites. Low bond: both ends below it;
// row = its row of the partner-position table. Crossing bond: low end lbit,
// high end hbit (in high coordinates); row = the table row of site lbit.
struct LoBondDev {
    uint32_t mask, row;
    double jz4, jxy2;
};
struct XBondDev {
    uint32_t hbit, row, lbit, pad;
    double jz4, jxy2;
};
struct SpinBlk {
    bool built = false, ok = false, f32 = false;
    int n_lo = 0, esize = 0, want = 0;
    int n_lob = 0, n_xb = 0, n_hib = 0;
    uint32_t n_blocks = 0, max_len = 0;
    std::unique_ptr<Species> sp;   // rank tables for this split point
    DevMem lob, xb, hib, tab, hi_list, cls_len, lo_off;
};

struct SpinSplit {
    bool built = false;
    int n_hi_bonds = 0, n_rest = 0;
    DevMem hib, rest, hi_list, cls_first, cls_len;
    std::vector<uint32_t> cls_first_h, cls_len_h;
    DevMem items[7];      // per positions per wave P = 2^i: per-XCD cumulative item counts
    bool items_ok[7] = {};
};

// SpinGC (full 2^N space): one off-diagonal term of a bit window. The
// tile index l holds the low bits and the window's bits; the term maps l to
// l ^ mloc with coefficient cpar when bits pi and pj of l agree, else canti
// (a field term has pi = pj).
struct GcTermDev {
    uint32_t mloc;
    uint32_t pi, pj;
    uint32_t pad;
    double cpar, canti;
};
struct GcDiagDev {
    uint32_t mask;   // (1 << i) | (1 << j)
    uint32_t pad;
    double jz4;      // jz / 4: +jz4 parallel, -jz4 antiparallel
};
// A plan of bit windows for one element size: window w takes the tile of
// 2^(lowb + q_w) states that vary in the low bits and its q_w window bits;
// the states of tile T have the complement bits set to the bits of T.
struct GcWindow {
    int q = 0;
    uint32_t wmask = 0, compmask = 0;
    size_t offw_first = 0;     // into GcPlan::offw (2^q entries)
    int term_first = 0, term_count = 0;
};
struct GcPlan {
    bool built = false;
    int lowb = 0;
    std::vector<GcWindow> wins;
    DevMem offw;    // uint32: scatter of the window index onto the window bits
    DevMem terms;   // GcTermDev
};

// Packed Hubbard neighbour entry: bits 0..23 target rank, 24..30 value
// class, bit 31 fermion sign.
constexpr uint32_t kNbrColMask = 0x00FFFFFFu;

// Value class 127 is reserved for 0.0: sliced-ELL padding entries point at
// their own column with that class, so padded slots need no branch.
constexpr uint32_t kZeroClass = 127u;
constexpr int kSellChunk = 64;

struct HubTables {
    DevMem off[2];   // uint32 [dim_sigma + 1]
    DevMem nbr[2];   // uint32 packed entries
    // sliced ELL of the same lists: chunks of 64 consecutive states, entry
    // k of state c at sell[base[c / 64] + k * 64 + c % 64], width[c / 64]
    // entries per state in the chunk (padded)
    DevMem sell_base[2], sell_width[2], sell[2];
    // Uniform |t| fast path (every transfer has the same magnitude t0):
    // lists split by fermion sign. Down species: sliced ELL of uint16
    // column indices, per chunk `plus` then `minus` widths, padded with the
    // index dim_dn (a zero slot). Up species: CSR with the sign split point.
    bool uniform_t = false;
    double t0 = 0.0;
    DevMem fs_base, fs_wp, fs_wm, fs_ent;    // down: chunk base, widths, uint16 entries
    DevMem fu_off, fu_mid, fu_ent;           // up: row offsets, split points, targets
    DevMem rr_off, rr_mid, rr_ent, rr_row;   // the same in reverse Cuthill-McKee row order; rr_row[p] = row
    // down species, hop-ordered slots (dim_dn < 32768): per chunk of 64
    // states one slot per hop active in any of them, in hop order, two slots
    // per uint32 (15-bit columns, signs in bits 31 and 30); inactive lanes
    // point at the zero slot dim_dn
    bool fb_ok = false;
    DevMem fb_base, fb_w, fb_ent;
    // the same slots with the low slot's LDS byte address pre-scaled
    // (element size 4 or 8: fc_ent[0] or [1]); built when dim_dn <= 16383
    bool fc_ok = false;
    DevMem fc_ent[2];
    // up species for the T_up tile kernel: blocks of consecutive rows
    // sharing the top ft_bits sites (rows ft_blk[b] .. ft_blk[b + 1]); by
    // position p (block-major, rows of a block in an order grouping equal hop
    // counts): ft_pos[p] the row's index in its block, ft_off[p] its first
    // entry, ft_cnt[p] four 8-bit counts (local plus, local minus, far plus,
    // far minus); entries: local = row index in the block, far = up row
    bool ft_ok = false;
    int ft_bits = 0, ft_nb = 0, ft_max_rows = 0;
    DevMem ft_blk, ft_pos, ft_off, ft_cnt, ft_ent;
    // two-body terms of the general Hamiltonian (exchange, pair hopping,
    // inter-site Coulomb, Hund): per-pair records and the same-species part
    // of their diagonal per up row and per down state (n_pairs = 0: none)
    int n_pairs = 0;
    DevMem pairs;                // HubPairDev [n_pairs]
    DevMem pair_eup, pair_edn;   // double [dim_up], [dim_dn]
    // per site k the pairs' other ends and V: the cross weights
    // m_k(u) = sum V u_other (site_off [n_sites + 1], site_nbr PairNbrDev)
    DevMem pair_site_off, pair_site_nbr;
    DevMem coef;     // double [128]: -t per value class (real parts)
    DevMem coef_im;  // double [128]: imaginary parts (complex transfers only)
    bool cplx = false;   // some transfer has an imaginary part: complex vectors only
    DevMem u_site;   // double [n_sites]
    int n_coef = 0;
    bool uniform_u = true;
    double u0 = 0.0;
    int64_t max_deg[2] = {0, 0};
};

// Time-dependent amplitudes of one Hubbard Hamiltonian: frames k = 0..n-1
// of the same terms, deduplicated per kind into slots (frames with equal
// values share one). The live tables of HubTables hold the slots in force;
// a frame switch copies a slot's tables over them on the caller's stream.
constexpr int kMaxFrames = 65536;
struct HubFrames {
    int n = 0, cur = 0;
    std::vector<int> hop_slot, u_slot, pair_slot;   // [n]
    int cur_hop = 0, cur_u = 0, cur_pair = 0;
    std::vector<double> hop_t;     // [hop slots][2][n_hops]: real parts, then imaginary parts
    std::vector<double> tau;       // [hop slots] t0 of the uniform-|t| path
    std::vector<double> u_site;    // [u slots][n_sites]
    std::vector<double> pair_v;    // [pair slots][n_pairs][4]: v, j_hund, j_ex, j_pair
    DevMem coef;                   // double [hop slots][256]: class values, real then imaginary
    DevMem u;                      // double [u slots][n_sites]
    DevMem pairs, nbr, eup, edn;   // per pair slot: records, site lists, same-species diagonals
    size_t nbr_n = 0;              // site-list entries per slot
};

} // namespace hphi

struct hphi_ham {
    hphi_basis *basis = nullptr;
    int kind = 0;
    // spin
    int n_bonds = 0;
    std::vector<hphi::SpinBondDev> bonds;
    hphi::DevMem d_bonds;
    hphi::DevMem d_hz;   // double [n_sites] or empty
    bool has_field = false;
    // Hubbard
    hphi::HubTables hub;
    std::vector<hphi_hop> hops;          // the terms, amplitudes of the frame in force
    std::vector<hphi_hop> hops_split;    // sign representatives of the uniform-|t| tables
    std::unique_ptr<hphi::HubFrames> td; // time-dependent amplitudes (null: fixed)
    std::vector<double> u_site;
    std::vector<hphi_pair_term> pair_terms;
    // SpinGC: XYZ bonds and fields, diagonal records, window plans per
    // element size (4, 8, 16 bytes per state)
    std::vector<hphi_xyz_bond> xyz;
    std::vector<double> hx, hz_gc;
    hphi::DevMem gc_diag, gc_hz;
    int gc_ndiag = 0;
    bool gc_has_hz = false;
    hphi::GcPlan gc_plan[3];
    // spin: bonds split into high-half and other bonds (built on first use)
    hphi::SpinSplit split;
    hphi::SpinBlk blk;
    bool noalloc_call = false;   // inside hphi_lanczos_noalloc
    // spin-S: bonds as given (jz, jxy), fields and single-ion terms
    std::vector<hphi_spin_bond> sbonds;
    std::vector<double> s_hz, s_dion;
    hphi::DevMem s_dbonds, s_dhz, s_ddion;
    // defaults: 128-column slabs, 128 workgroups per XCD, 32-row items,
    // hop-ordered down slots, work-item queues with two columns per lane;
    // spin: 8 workgroups per CU
    hphi_schedule sched_cfg{128, 128, 16, 6, 8, 0, 5, 2, 0, 0, 3, 0};
    // scratch for reductions and work queues
    hphi::DevMem sched;         // unsigned [16]: per-XCD item queues + counter
    hphi::DevMem red_partial;   // double [kReduceSlots]
    hphi::DevMem red_counter;   // unsigned [16]
    hphi::DevMem red_result;    // double [64]
    // one call at a time, one stream at a time (the scratch above is shared)
    hphi::UseState use;
    hphi_ham() = default;
    hphi_ham(const hphi_ham &) = delete;
    hphi_ham &operator=(const hphi_ham &) = delete;
    ~hphi_ham()
    {
        if (use.event) (void)hipEventDestroy((hipEvent_t)use.event);
    }
};

namespace hphi {

// The guard's device side: an event recorded at the end of each call.
struct HipUseOps {
    bool pending(void *e) { return hipEventQuery((hipEvent_t)e) == hipErrorNotReady; }
    void record(void *e, void *st) { (void)hipEventRecord((hipEvent_t)e, (hipStream_t)st); }
    bool capturing(void *st)
    {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing((hipStream_t)st, &cs) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        return cs != hipStreamCaptureStatusNone;
    }
};

struct HamUse {
    HipUseOps ops;
    UseScope<HipUseOps> scope;
    HamUse(hphi_ham *h, void *st) : scope(h->use, ops, st) {}
};

// Creates the Hamiltonian's guard event (after its device is current).
int init_ham_use(hphi_ham *h);
// reduction and queue scratch of a Hamiltonian (allocated once)
int ham_ensure_reduce(hphi_ham *h);
// time-dependent amplitudes: puts frame k in force on stream st
int ham_apply_frame(hphi_ham *h, int k, hipStream_t st);

} // namespace hphi

// A non-blocking stream for work that must be captured into a graph when
// the caller gave the legacy default stream (which cannot be captured); the
// default stream's queued work is waited for first. Synchronized and
// destroyed at scope exit.
struct OwnStream {
    hipStream_t s = nullptr;
    int make(hipStream_t *st)
    {
        HPHI_HIP(hipStreamSynchronize(nullptr));
        HPHI_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
        *st = s;
        return HPHI_OK;
    }
    ~OwnStream()
    {
        if (s) {
            (void)hipStreamSynchronize(s);
            (void)hipStreamDestroy(s);
        }
    }
};

// Enter a call on Hamiltonian h issued on stream st (after the device guard);
// returns HPHI_ERR_BUSY from the enclosing function when it may not start.
#define HPHI_USE_HAM(h, st)                                                                    \
    ::hphi::HamUse hphi_use_((h), (void *)(st));                                               \
    if (hphi_use_.scope.verdict() != ::hphi::USE_OK)                                           \
        return ::hphi::fail(HPHI_ERR_BUSY, "%s",                                               \
                            hphi_use_.scope.verdict() == ::hphi::USE_OTHER_THREAD              \
                                ? "the Hamiltonian is in a call on another thread"             \
                                : "the previous call on this Hamiltonian still runs on another stream")

namespace hphi {

constexpr int kMaxGrid = 4096;
constexpr int64_t kReduceSlots = int64_t(1) << 20;   // doubles of reduction scratch

// Reduction target: per-block partial sums, a completion counter, and the
// reduced result (first `n` doubles) written by the last block to finish.
struct Reduce {
    double *partial = nullptr;
    unsigned *counter = nullptr;
    double *result = nullptr;
};

// ---- kernel launchers (kernels.hip) ----
// w = c1 * (H v) + c2 * u; coef = device [c1, c2] or nullptr (c1 = 1, c2 = 0);
// u may be nullptr. dots: 0 = none, 1 = sum v.w per lane, 2 = v.w and w.w
// per lane (result[lane], result[nlanes + lane]).
struct MultArgs {
    int dtype;          // hphi_dtype
    int nvec;           // vectors in the block
    const void *v;
    void *w;
    const void *u;
    void *acc;          // optional: acc += w (same layout)
    const double *coef;
    int dots;           // 0: none; 1: per-lane <v, x> and <x, x>
    int dot_raw;        // x = H v (1) or x = the epilogue output w (0)
    Reduce red;
    hipStream_t stream;
    int coef_cplx;      // coef = [c1 re, c2 re, c1 im, c2 im] applied to complex pairs
    // Lanczos update of the previous step fused into the product (Hubbard
    // rows kernel; only where hub_rows_fused_ok): v <- v - f lz_q first
    struct LzDev *lz;
    double *lz_alpha, *lz_beta;
    const void *lz_q;
    Reduce lz_red;
    hipEvent_t ev_mid;  // optional: recorded between the two kernels of a Hubbard H*v
    void *raw_out;      // optional (spin, stored basis): H v before the epilogue
    void *cocg;         // optional (spin, stored basis, one complex vector, dots = 1):
                        // the dots become the COCG mu = v^T (z_s v - H v) and the
                        // last block does the alpha step on this CgDev
    int64_t ld;         // Hubbard: row pitch of v, w, u, lz_q in elements (0: dim_dn)
};
bool hub_rows_fused_ok(hphi_ham *h, int nv);
bool spin_stored_path(const hphi_ham *h);
// Spin product layout for the schedule in force: 0 one pass, 1 two passes
// by bond locality, 2 block-staged (implicit basis). spin_split 3 (the
// default) means 2 on the implicit basis and one pass on the stored list;
// calls that must not allocate take one pass (the other layouts build
// device tables on first use).
int spin_split_mode(const hphi_ham *h, bool implicit);
int launch_spin_mult(hphi_ham *h, const MultArgs &a);
int launch_spin_mult_implicit(hphi_ham *h, const MultArgs &a);
int spin_split_tables(hphi_ham *h);
int launch_spin_hi_pass(hphi_ham *h, const MultArgs &a);
// Block-staged product on the implicit basis: builds its tables on first use
// for an element size; sets *done when it ran (0: the blocks do not fit LDS
// at any split point, the caller takes another path)
int launch_spin_blk(hphi_ham *h, const MultArgs &a, int *done);
int launch_hub_mult(hphi_ham *h, const MultArgs &a);
int launch_mult(hphi_ham *h, const MultArgs &a);
// w += H_2body v for the Hubbard two-body terms (NV lanes per element, rows
// of pitch ld elements); a no-op without pair terms
int launch_hub_pairs(hphi_ham *h, int elem_bytes, int nv, const void *v, void *w, int64_t ld, hipStream_t st);
// SpinGC: H*v by bit windows, the diagonal, the trace, S^z(q), states/ranks
int launch_gc_mult(hphi_ham *h, const MultArgs &a);
int gc_plan_build(hphi_ham *h, int esz_index);
int launch_gc_diag(hphi_ham *h, double *out, hipStream_t st);
int launch_gc_trace(hphi_ham *h, Reduce red, hipStream_t st);
int launch_gc_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st);
int launch_gc_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out, hipStream_t st);
int launch_gc_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx, hipStream_t st);
// spin-S: H*v, the diagonal, the trace, S^z(q), states/ranks
int launch_spin_s_mult(hphi_ham *h, const MultArgs &a);
int launch_spin_s_diag(hphi_ham *h, double *out, hipStream_t st);
int launch_spin_s_trace(hphi_ham *h, Reduce red, hipStream_t st);
int launch_spin_s_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st);
int launch_spin_s_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out, hipStream_t st);
int launch_spin_s_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx, hipStream_t st);

int launch_rank_device(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx,
                       hipStream_t st);
int launch_states_device(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out,
                         hipStream_t st);
int launch_materialize(Species &s, hipStream_t st);

// vector kernels
int launch_rng_uniform(int dtype, void *out, int64_t n, uint64_t seed, hipStream_t st);
int launch_rng_cgauss(int dtype, void *out, int64_t dim, int nvec, uint64_t seed, hipStream_t st);
int launch_dots(int dtype, int nlanes, int64_t rows, const void *x, const void *y, Reduce red,
                int mode, hipStream_t st);   // mode 0: x.y per lane; 1: x.x per lane
// x.y per lane into result[lane] and y.y into result[nlanes + lane]; one
// thread per scalar of the flat [rows][nlanes] arrays (nlanes divides 256)
int launch_dots_xy_yy(int dtype, int nlanes, int64_t rows, const void *x, const void *y, Reduce red,
                      hipStream_t st);
int launch_scale_lanes(int dtype, int nlanes, int64_t rows, void *x, const double *scale_dev,
                       int mode, hipStream_t st);   // mode 0: x *= s[lane]; 1: x *= 1/sqrt(s[lane])
int launch_axpy_lanes(int dtype, int nlanes, int64_t rows, void *y, const void *x,
                      const double *a_dev, double a_host, hipStream_t st);
int launch_copy_cast(int dst_dtype, void *dst, int src_dtype, const void *src, int64_t n,
                     hipStream_t st);
int launch_trace(hphi_ham *h, Reduce red, hipStream_t st);
int launch_docc(hphi_ham *h, int dtype, const void *psi, Reduce red, hipStream_t st);
int launch_szq(hphi_ham *h, const double *phase_dev, const void *psi, void *b, hipStream_t st);

// Lanczos device scalars and kernels
struct LzDev {
    double coef[2];      // H*v epilogue: c1 = s_k, c2 = -beta_k s_{k-1}
    double dot[4];       // result slot of the H*v kernel's <q_k, w>
    double nrm[4];       // result slot of the update kernel / initial norm
    double s_cur, s_prev;
    double psi_coef;     // second pass: coefficient of q_k in psi
    int iter;
    int done;
    int breakdown;
    int pad;
};
int launch_lz_init(int dtype, LzDev *lz, int64_t dim, Reduce red, hipStream_t st);
int launch_lz_update(int dtype, LzDev *lz, double *alpha, double *beta, int64_t dim, void *w,
                     const void *qk, Reduce red, hipStream_t st);
// q stored in rows of `cols` elements at pitch ld (cols = 0: unpadded)
int launch_lz_psi_accum(int psi_dtype, int dtype, LzDev *lz, const double *svec, int64_t dim, void *psi,
                        const void *qk, hipStream_t st, int64_t cols = 0, int64_t ld = 0);
int launch_rng_uniform_pitched(int dtype, void *out, int64_t rows, int64_t cols, int64_t ld, uint64_t seed,
                               hipStream_t st);
int launch_norm2_pitched(int dtype, const void *x, int64_t dim, int64_t cols, int64_t ld, Reduce red, hipStream_t st);
// dst[counter[which] * row + i] = src[i] for i < n; counter[which]++ (one step's results per row)
int launch_record(const double *src, int n, double *dst, int row, int *counter, int which, hipStream_t st);
// Row pitch (elements) a Hubbard Lanczos run may store its vectors with
// (rows padded to whole 128-byte lines) for the current schedule; dim_dn
// when the kernels it selects take only unpadded rows.
int64_t hub_lanczos_pitch(hphi_ham *h, int dtype);

// Static device scratch of the no-allocation Lanczos entry point
// (noalloc.hip): set up per device in hphi_init; one call at a time per
// device (acquire returns HPHI_ERR_BUSY otherwise).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
int noalloc_scratch_init(int device);
int noalloc_scratch_acquire(int device, void **ptr);
void noalloc_scratch_release(int device);
// zero fill by a kernel (bytes a multiple of 4, 4-byte aligned)
int launch_zero(void *p, size_t bytes, hipStream_t st);

// host tridiagonal solver
int tridiag_lowest(const double *alpha, const double *beta, int n, int k, double *eig,
                   double *vec);

// The Hamiltonian's reduction scratch with the result written to `result`.
inline Reduce reduce_at(hphi_ham *h, double *result)
{
    Reduce r;
    r.partial = h->red_partial.as<double>();
    r.counter = h->red_counter.as<unsigned>();
    r.result = result;
    return r;
}

int dtype_size(int dtype);     // bytes per scalar element (complex counts 2 lanes)
int dtype_lanes(int dtype);    // 1 real, 2 complex
bool dtype_is_f32(int dtype);

} // namespace hphi

namespace hphi {

// ---- shifted COCG state (kern_methods.hip) ----
struct cd {
    double re, im;
};

struct CgDev {
    cd zs;
    cd rho;                 // r_k^T r_k
    cd alpha, beta;         // current alpha_k, beta_k
    cd alpha_prev, beta_prev;
    double rnorm2;          // |r_{k+1}|^2
    double bnorm2;          // |b|^2
    cd bhr;                 // b^H r_{k+1}
    double max_res;         // max over unconverged shifts of |r_j| / |b|
    int iter;
    int breakdown;
};

struct ShiftDev {
    cd sigma, pi, pi_prev, X, P;
    double res;
    int conv;
    int pad;
};

int launch_cocg_init(const void *b, void *r, void *p, int64_t dim, void *cg, void *sh, int nsh, double tol,
                     Reduce red, hipStream_t st);
int launch_cocg_iter(void *r, void *p, const void *h, const void *b, int64_t dim, void *cg, void *sh,
                     int nsh, double tol, Reduce red, hipStream_t st, bool mu_done = false);
int launch_cplx_part(const void *b, void *out, int64_t dim, int part, hipStream_t st);
int launch_pair_rsqrt(const double *n, double *s, int nl, hipStream_t st);

// batched S(q, w): one shifted-COCG sequence per workgroup (kern_batch.hip)
size_t cocg_item_size();
int64_t cocg_chunks(int64_t dim);
int fill_cocg_item(hphi_ham *h, const void *b, int part, double *r, double *p, double *hv, double *chunks,
                   void *sh, int nsh, double zs_re, double zs_im, double tol, int max_iter, double *out, void *dst);
int launch_cocg_batch(const void *items_dev, int n, hipStream_t st);

// batched small-sector Lanczos (kern_batch.hip)
size_t batch_item_size();
int fill_batch_item(hphi_ham *h, int iters, uint64_t seed, double *q, double *alpha, double *beta, int *done,
                    double *part, unsigned *bar, int team_base, void *out);
int launch_lanczos_team(const void *items_dev, int n, int grid, unsigned *ticket, hipStream_t st);
size_t batch_part_doubles(int64_t dim);
void batch_team_shape(int64_t dim, int *w, int *rows);
int launch_lanczos_batch(const void *items_dev, int n, hipStream_t st, size_t lds_bytes);
size_t batch_lds_bytes(int64_t dim, int n_lo, int n_hi);

} // namespace hphi

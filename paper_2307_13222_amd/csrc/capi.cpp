// C ABI entry points: contexts, bases, Hamiltonians, H*v, trace, Lanczos.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>

#include <cstdio>
#include <cstdlib>

#include "internal.h"

using namespace hphi;

namespace {


int ensure_reduce(hphi_ham *h)
{
    if (!h->red_partial.p) {
        HPHI_TRY(h->red_partial.alloc(sizeof(double) * (size_t)kReduceSlots));
        HPHI_TRY(h->red_counter.alloc(sizeof(unsigned) * 16));
        HPHI_TRY(zero_now(h->red_counter.p, sizeof(unsigned) * 16));
        HPHI_TRY(h->sched.alloc(sizeof(unsigned) * 16));
        HPHI_TRY(zero_now(h->sched.p, sizeof(unsigned) * 16));
        HPHI_TRY(h->red_result.alloc(sizeof(double) * 128));
    }
    return init_ham_use(h);
}

Reduce reduce_of(hphi_ham *h, double *result = nullptr)
{
    Reduce r;
    r.partial = h->red_partial.as<double>();
    r.counter = h->red_counter.as<unsigned>();
    r.result = result ? result : h->red_result.as<double>();
    return r;
}

} // namespace

namespace hphi {

int init_ham_use(hphi_ham *h)
{
    if (h->use.event) return HPHI_OK;
    hipEvent_t e = nullptr;
    HPHI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    h->use.event = (void *)e;
    return HPHI_OK;
}

int ham_ensure_reduce(hphi_ham *h) { return ensure_reduce(h); }

int launch_mult(hphi_ham *h, const MultArgs &a)
{
    if (h->kind == 0) return launch_spin_mult(h, a);
    if (h->kind == 2) return launch_gc_mult(h, a);
    if (h->kind == 3) return launch_spin_s_mult(h, a);
    return launch_hub_mult(h, a);
}

} // namespace hphi

extern "C" {

const char *hphi_version(void) { return "hphi_mi355 0.1 (gfx950)"; }

const char *hphi_last_error(void) { return hphi::last_error(); }

int hphi_init(int device, hphi_ctx **ctx)
{
    if (!ctx) return fail(HPHI_ERR_INVALID_ARG, "ctx is NULL");
    int n = 0;
    HPHI_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(HPHI_ERR_INVALID_ARG, "device %d of %d", device, n);
    HPHI_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    HPHI_HIP(hipGetDeviceProperties(&prop, device));
    auto *c = new hphi_ctx;
    c->device = device;
    c->n_cu = prop.multiProcessorCount;
    c->lds_per_block = prop.sharedMemPerBlock;
    const int rc = noalloc_scratch_init(device);
    if (rc != HPHI_OK) {
        delete c;
        return rc;
    }
    *ctx = c;
    return HPHI_OK;
}

void hphi_fini(hphi_ctx *ctx) { delete ctx; }

int hphi_basis_spin(hphi_ctx *ctx, int n_sites, int two_sz, hphi_basis **out)
{
    if (!ctx || !out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (n_sites < 1 || n_sites > 64) return fail(HPHI_ERR_INVALID_ARG, "n_sites %d outside [1, 64]", n_sites);
    if (std::abs(two_sz) > n_sites || ((n_sites + two_sz) & 1))
        return fail(HPHI_ERR_INVALID_ARG, "2Sz = %d impossible for %d sites", two_sz, n_sites);
    DeviceGuard g(ctx->device);
    std::unique_ptr<hphi_basis> b(new hphi_basis);
    b->ctx = ctx;
    b->kind = 0;
    b->n_sites = n_sites;
    const int n_up = (n_sites + two_sz) / 2;
    // materialize the state list when it is addressable by 32-bit indices
    // and configurations fit 32 bits; larger sectors stay implicit
    const bool mat = n_sites <= 32;
    HPHI_TRY(build_species(b->sp[0], n_sites, n_up, 0, false));
    if (mat && b->sp[0].dim < (int64_t(1) << 32)) {
        HPHI_TRY(b->sp[0].d_states.alloc((size_t)b->sp[0].dim * b->sp[0].state_bytes));
        HPHI_TRY(launch_materialize(b->sp[0], nullptr));
        HPHI_HIP(hipDeviceSynchronize());
    }
    b->dim = b->sp[0].dim;
    *out = b.release();
    return HPHI_OK;
}

int hphi_basis_hubbard(hphi_ctx *ctx, int n_sites, int n_up, int n_dn, hphi_basis **out)
{
    if (!ctx || !out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (n_sites < 1 || n_sites > 32) return fail(HPHI_ERR_INVALID_ARG, "n_sites %d outside [1, 32]", n_sites);
    if (n_up < 0 || n_up > n_sites || n_dn < 0 || n_dn > n_sites)
        return fail(HPHI_ERR_INVALID_ARG, "n_up/n_dn outside [0, %d]", n_sites);
    DeviceGuard g(ctx->device);
    std::unique_ptr<hphi_basis> b(new hphi_basis);
    b->ctx = ctx;
    b->kind = 1;
    b->n_sites = n_sites;
    HPHI_TRY(build_species(b->sp[0], n_sites, n_up, 0, true));
    HPHI_TRY(build_species(b->sp[1], n_sites, n_dn, 0, true));
    if (b->sp[0].dim > (int64_t)kNbrColMask || b->sp[1].dim > (int64_t)kNbrColMask)
        return fail(HPHI_ERR_DIM_OVERFLOW, "one-species dimension above 2^24");
    unsigned __int128 d = (unsigned __int128)b->sp[0].dim * (unsigned __int128)b->sp[1].dim;
    if (d > ((unsigned __int128)1 << 62)) return fail(HPHI_ERR_DIM_OVERFLOW, "dimension beyond 2^62");
    b->dim = (int64_t)d;
    *out = b.release();
    return HPHI_OK;
}

void hphi_basis_free(hphi_basis *b) { delete b; }

int64_t hphi_basis_dim(const hphi_basis *b) { return b ? b->dim : 0; }

int hphi_basis_states(const hphi_basis *b, int64_t first, int64_t count, uint64_t *host_out)
{
    if (!b || (!host_out && count > 0)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (first < 0 || count < 0 || first + count > b->dim) return fail(HPHI_ERR_INVALID_ARG, "range outside the basis");
    for (int64_t t = 0; t < count; ++t) {
        const int64_t r = first + t;
        if (b->kind == 2) {
            host_out[t] = (uint64_t)r;
        } else if (b->kind == 3) {
            host_out[t] = b->ss.states[(size_t)r];
        } else if (b->kind == 0) {
            host_out[t] = b->sp[0].state_at(r);
        } else {
            const int64_t ru = r / b->sp[1].dim, rd = r % b->sp[1].dim;
            host_out[t] = (b->sp[0].state_at(ru) << 32) | b->sp[1].state_at(rd);
        }
    }
    return HPHI_OK;
}

int hphi_basis_rank(const hphi_basis *b, const uint64_t *states, int64_t n, int64_t *idx_out)
{
    if (!b || ((!states || !idx_out) && n > 0)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    for (int64_t t = 0; t < n; ++t) {
        if (b->kind == 2) {
            idx_out[t] = states[t] < (uint64_t)b->dim ? (int64_t)states[t] : -1;
        } else if (b->kind == 3) {
            idx_out[t] = b->ss.rank_of(states[t]);
        } else if (b->kind == 0) {
            idx_out[t] = b->sp[0].rank_of(states[t]);
        } else {
            const int64_t ru = b->sp[0].rank_of(states[t] >> 32);
            const int64_t rd = b->sp[1].rank_of(states[t] & 0xFFFFFFFFull);
            idx_out[t] = (ru < 0 || rd < 0) ? -1 : ru * b->sp[1].dim + rd;
        }
    }
    return HPHI_OK;
}

int hphi_basis_states_device(const hphi_basis *b, int64_t first, int64_t count, uint64_t *out_dev, void *stream)
{
    if (!b || (!out_dev && count > 0)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (first < 0 || count < 0 || first + count > b->dim) return fail(HPHI_ERR_INVALID_ARG, "range outside the basis");
    DeviceGuard g(b->ctx->device);
    if (b->kind == 2) return launch_gc_states(b, first, count, out_dev, (hipStream_t)stream);
    if (b->kind == 3) return launch_spin_s_states(b, first, count, out_dev, (hipStream_t)stream);
    return launch_states_device(b, first, count, out_dev, (hipStream_t)stream);
}

int hphi_basis_rank_device(const hphi_basis *b, const uint64_t *states_dev, int64_t n, int64_t *idx_dev, void *stream)
{
    if (!b || ((!states_dev || !idx_dev) && n > 0) || n < 0) return fail(HPHI_ERR_INVALID_ARG, "bad argument");
    DeviceGuard g(b->ctx->device);
    if (b->kind == 2) return launch_gc_rank(b, states_dev, n, idx_dev, (hipStream_t)stream);
    if (b->kind == 3) return launch_spin_s_rank(b, states_dev, n, idx_dev, (hipStream_t)stream);
    return launch_rank_device(b, states_dev, n, idx_dev, (hipStream_t)stream);
}

int hphi_basis_tables(const hphi_basis *b, int species, const uint32_t **lo_rank, const uint64_t **hi_off,
                      int *n_lo, int *n_hi)
{
    if (b && b->kind >= 2) return fail(HPHI_ERR_UNSUPPORTED, "SpinGC and spin-S bases have no species tables");
    if (!b || species < 0 || species > b->kind) return fail(HPHI_ERR_INVALID_ARG, "bad species");
    const Species &s = b->sp[species];
    if (lo_rank) *lo_rank = s.lo_rank.data();
    if (hi_off) *hi_off = s.hi_off.data();
    if (n_lo) *n_lo = s.n_lo;
    if (n_hi) *n_hi = s.n_hi;
    return HPHI_OK;
}

int hphi_ham_spin(hphi_basis *b, const hphi_spin_bond *bonds, int n_bonds, const double *hz, hphi_ham **out)
{
    if (!b || !out || (n_bonds > 0 && !bonds)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (b->kind != 0) return fail(HPHI_ERR_INVALID_ARG, "spin Hamiltonian needs a spin basis");
    if (n_bonds < 0 || n_bonds > 4096) return fail(HPHI_ERR_INVALID_ARG, "n_bonds %d outside [0, 4096]", n_bonds);
    DeviceGuard g(b->ctx->device);
    std::unique_ptr<hphi_ham> h(new hphi_ham);
    h->basis = b;
    h->kind = 0;
    h->n_bonds = n_bonds;
    for (int k = 0; k < n_bonds; ++k) {
        const int i = bonds[k].i, j = bonds[k].j;
        if (i < 0 || j < 0 || i >= b->n_sites || j >= b->n_sites || i == j)
            return fail(HPHI_ERR_INVALID_ARG, "bond %d (%d, %d) invalid for %d sites", k, i, j, b->n_sites);
        SpinBondDev d{};
        d.mask = (uint64_t(1) << i) | (uint64_t(1) << j);
        d.jz4 = 0.25 * bonds[k].jz;
        d.jxy2 = 0.5 * bonds[k].jxy;
        d.i = i;
        d.j = j;
        h->bonds.push_back(d);
    }
    if (n_bonds > 0) HPHI_TRY(upload(h->d_bonds, h->bonds.data(), sizeof(SpinBondDev) * n_bonds));
    else HPHI_TRY(h->d_bonds.alloc(sizeof(SpinBondDev)));
    if (hz) {
        h->has_field = true;
        HPHI_TRY(upload(h->d_hz, hz, sizeof(double) * b->n_sites));
    }
    HPHI_TRY(ensure_reduce(h.get()));
    *out = h.release();
    return HPHI_OK;
}

// Per-species neighbour lists of the hopping matrix T_sigma: for state s
// and transfer (i, j) with exactly one of i, j occupied, the target
// s ^ (1<<i | 1<<j), value -t and sign (-1)^(occupied sites strictly
// between i and j).
// hop_cls_i / hop_cls_j: value class of hop k in a row whose state holds
// site i / site j of the hop (the same class for real transfers)
static int build_hub_species(const Species &sp, const std::vector<hphi_hop> &hops,
                             const std::vector<int> &hop_cls_i, const std::vector<int> &hop_cls_j, DevMem &off_d,
                             DevMem &nbr_d, int64_t &max_deg,
                             DevMem &sell_base_d, DevMem &sell_width_d, DevMem &sell_d)
{
    std::vector<uint32_t> off((size_t)sp.dim + 1, 0);
    std::vector<uint32_t> ent;
    ent.reserve((size_t)sp.dim * hops.size() / 2 + 1);
    max_deg = 0;
    for (int64_t r = 0; r < sp.dim; ++r) {
        const uint64_t s = sp.state_at(r);
        off[r] = (uint32_t)ent.size();
        for (size_t hk = 0; hk < hops.size(); ++hk) {
            const hphi_hop &hp = hops[hk];
            const int bi = (int)((s >> hp.i) & 1), bj = (int)((s >> hp.j) & 1);
            if (bi == bj) continue;
            const uint64_t t = s ^ ((uint64_t(1) << hp.i) | (uint64_t(1) << hp.j));
            const int lo = std::min(hp.i, hp.j), hi = std::max(hp.i, hp.j);
            const uint64_t between = (hi - lo > 1) ? (((uint64_t(1) << hi) - 1) & ~((uint64_t(1) << (lo + 1)) - 1)) : 0;
            const uint32_t sign = (uint32_t)(__builtin_popcountll(s & between) & 1);
            const int64_t tr = sp.rank_of(t);
            const int cls = bi ? hop_cls_i[hk] : hop_cls_j[hk];
            ent.push_back((uint32_t)tr | ((uint32_t)cls << 24) | (sign << 31));
        }
        max_deg = std::max<int64_t>(max_deg, (int64_t)ent.size() - off[r]);
        if (ent.size() > 0xFFFFFFF0ull) return fail(HPHI_ERR_DIM_OVERFLOW, "neighbour list above 2^32 entries");
    }
    off[sp.dim] = (uint32_t)ent.size();
    // sliced ELL, padded with zero-valued self entries
    const int64_t nchunk = (sp.dim + kSellChunk - 1) / kSellChunk;
    std::vector<uint32_t> base(nchunk + 1, 0), width(nchunk, 0), sell;
    for (int64_t j = 0; j < nchunk; ++j) {
        uint32_t wmax = 0;
        for (int64_t c = j * kSellChunk; c < std::min(sp.dim, (j + 1) * kSellChunk); ++c)
            wmax = std::max(wmax, off[c + 1] - off[c]);
        width[j] = wmax;
        base[j + 1] = base[j] + wmax * kSellChunk;
    }
    sell.assign(base[nchunk] > 0 ? base[nchunk] : 1, 0u);
    for (int64_t j = 0; j < nchunk; ++j)
        for (int l = 0; l < kSellChunk; ++l) {
            const int64_t c = j * kSellChunk + l;
            for (uint32_t k = 0; k < width[j]; ++k) {
                uint32_t e = (uint32_t)(c < sp.dim ? c : 0) | (kZeroClass << 24);
                if (c < sp.dim && k < off[c + 1] - off[c]) e = ent[off[c] + k];
                sell[base[j] + (size_t)k * kSellChunk + l] = e;
            }
        }
    HPHI_TRY(upload(off_d, off.data(), sizeof(uint32_t) * off.size()));
    if (ent.empty()) ent.push_back(0);
    HPHI_TRY(upload(nbr_d, ent.data(), sizeof(uint32_t) * ent.size()));
    HPHI_TRY(upload(sell_base_d, base.data(), sizeof(uint32_t) * base.size()));
    HPHI_TRY(upload(sell_width_d, width.data(), sizeof(uint32_t) * width.size()));
    HPHI_TRY(upload(sell_d, sell.data(), sizeof(uint32_t) * sell.size()));
    return HPHI_OK;
}

// Neighbour lists of one species split by the sign of the matrix element
// -t_h * (-1)^(occupied sites between): with all |t_h| = t0 the element is
// -t0 * s, s = sign(t_h) * fermion sign; `plus` holds s = +1, `minus` s = -1.
static void split_lists(const Species &sp, const std::vector<hphi_hop> &hops,
                        std::vector<std::vector<uint32_t>> &plus, std::vector<std::vector<uint32_t>> &minus)
{
    plus.assign((size_t)sp.dim, {});
    minus.assign((size_t)sp.dim, {});
    for (int64_t r = 0; r < sp.dim; ++r) {
        const uint64_t s = sp.state_at(r);
        for (const hphi_hop &hp : hops) {
            if (((s >> hp.i) & 1) == ((s >> hp.j) & 1)) continue;
            const uint64_t t = s ^ ((uint64_t(1) << hp.i) | (uint64_t(1) << hp.j));
            const int lo = std::min(hp.i, hp.j), hi = std::max(hp.i, hp.j);
            const uint64_t between = (hi - lo > 1) ? (((uint64_t(1) << hi) - 1) & ~((uint64_t(1) << (lo + 1)) - 1)) : 0;
            const int fs = (__builtin_popcountll(s & between) & 1) ? -1 : 1;
            const int se = fs * (hp.t < 0 ? -1 : 1);
            (se > 0 ? plus : minus)[r].push_back((uint32_t)sp.rank_of(t));
        }
    }
}

// Reverse Cuthill-McKee order of an undirected graph given by adjacency
// lists (Cuthill and McKee 1969; reversed as George recommends): level-order
// traversal from a pseudo-peripheral node, each node's unvisited neighbours
// taken by increasing degree, a new start per connected component, then the
// whole sequence reversed. The start node comes from repeated breadth-first
// passes (George and Liu): from a node of least degree, move to a node of
// least degree in the last level while the number of levels grows.
static std::vector<uint32_t> rcm_order(const std::vector<std::vector<uint32_t>> &adj)
{
    const size_t n = adj.size();
    std::vector<uint32_t> order;
    order.reserve(n);
    std::vector<char> seen(n, 0);
    std::vector<int> level(n, -1);
    auto deg = [&](uint32_t x) { return adj[x].size(); };
    // levels of a breadth-first pass restricted to unseen nodes
    auto bfs_levels = [&](uint32_t s, std::vector<uint32_t> &last) {
        std::vector<uint32_t> cur{s}, touched{s};
        level[s] = 0;
        int depth = 0;
        last = cur;
        while (!cur.empty()) {
            std::vector<uint32_t> nxt;
            for (uint32_t x : cur)
                for (uint32_t y : adj[x])
                    if (!seen[y] && level[y] < 0) {
                        level[y] = depth + 1;
                        nxt.push_back(y);
                        touched.push_back(y);
                    }
            if (!nxt.empty()) last = nxt;
            cur.swap(nxt);
            if (!cur.empty()) ++depth;
        }
        for (uint32_t x : touched) level[x] = -1;
        return depth;
    };
    for (size_t c0 = 0; c0 < n; ++c0) {
        if (seen[c0]) continue;
        // least-degree unseen node of this component as the first guess
        uint32_t s = (uint32_t)c0;
        {
            std::vector<uint32_t> stack{s};
            std::vector<uint32_t> mark;
            level[s] = 0;
            mark.push_back(s);
            while (!stack.empty()) {
                const uint32_t x = stack.back();
                stack.pop_back();
                if (deg(x) < deg(s)) s = x;
                for (uint32_t y : adj[x])
                    if (!seen[y] && level[y] < 0) {
                        level[y] = 0;
                        mark.push_back(y);
                        stack.push_back(y);
                    }
            }
            for (uint32_t x : mark) level[x] = -1;
        }
        std::vector<uint32_t> last;
        int ecc = bfs_levels(s, last);
        for (int guard = 0; guard < 16; ++guard) {
            uint32_t best = last[0];
            for (uint32_t x : last)
                if (deg(x) < deg(best)) best = x;
            std::vector<uint32_t> last2;
            const int e2 = bfs_levels(best, last2);
            if (e2 <= ecc) break;
            s = best;
            ecc = e2;
            last.swap(last2);
        }
        // Cuthill-McKee from s
        const size_t first = order.size();
        order.push_back(s);
        seen[s] = 1;
        for (size_t k = first; k < order.size(); ++k) {
            std::vector<uint32_t> nb;
            for (uint32_t y : adj[order[k]])
                if (!seen[y]) {
                    seen[y] = 1;
                    nb.push_back(y);
                }
            std::stable_sort(nb.begin(), nb.end(), [&](uint32_t a, uint32_t b) { return deg(a) < deg(b); });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// Tile tables of the up species (see HubTables::ft_*): blocks of consecutive
// up rows sharing the top `bits` sites; each row's hops split into local
// (target in the block: row index in the block) and far (target row), each
// by fermion sign; the rows of a block ordered by (far count, local count)
// so the eight rows of a wave walk lists of similar length. bits = 0: the
// fewest top sites whose largest block fits the kernel's LDS in FP64. Sets
// ft_ok false when the shape does not fit the kernel.
constexpr int kTileMaxRowsF64 = 1135;   // (160 KiB - reduction scratch) / 144-byte rows

static int build_hub_tile(hphi_ham *h, int bits)
{
    HubTables &T = h->hub;
    T.ft_ok = false;
    const Species &up = h->basis->sp[0];
    if (!T.uniform_t || up.dim >= (int64_t(1) << 24) || up.n_bits > 32) return HPHI_OK;
    const int n = up.n_bits;
    auto block_starts = [&](int nb_bits) {
        std::vector<uint32_t> blk;
        uint64_t prev = ~uint64_t(0);
        for (int64_t r = 0; r < up.dim; ++r) {
            const uint64_t lab = nb_bits > 0 ? up.state_at(r) >> (n - nb_bits) : 0;
            if (lab != prev) {
                blk.push_back((uint32_t)r);
                prev = lab;
            }
        }
        blk.push_back((uint32_t)up.dim);
        return blk;
    };
    auto max_rows = [](const std::vector<uint32_t> &blk) {
        uint32_t m = 0;
        for (size_t b = 0; b + 1 < blk.size(); ++b) m = std::max(m, blk[b + 1] - blk[b]);
        return m;
    };
    std::vector<uint32_t> blk;
    if (bits <= 0) {
        for (bits = 1; bits <= n; ++bits) {
            blk = block_starts(bits);
            if (max_rows(blk) <= (uint32_t)kTileMaxRowsF64) break;
        }
        if (bits > n) return HPHI_OK;
    } else {
        if (bits > n) return fail(HPHI_ERR_INVALID_ARG, "hub_tile_bits %d above the site count", bits);
        blk = block_starts(bits);
        if (max_rows(blk) > (uint32_t)kTileMaxRowsF64) {
            T.ft_bits = bits;
            return HPHI_OK;
        }
    }
    std::vector<std::vector<uint32_t>> pl, mi;
    split_lists(up, h->hops_split, pl, mi);
    const size_t nb = blk.size() - 1;
    std::vector<uint32_t> pos((size_t)up.dim), off((size_t)up.dim + 1, 0), cnt((size_t)up.dim), ent;
    bool ok = true;
    for (size_t b = 0; b < nb; ++b) {
        const uint32_t b0 = blk[b], b1 = blk[b + 1];
        std::vector<uint32_t> rows(b1 - b0);
        std::vector<uint32_t> nloc(b1 - b0), nfar(b1 - b0);
        for (uint32_t r = b0; r < b1; ++r) {
            rows[r - b0] = r - b0;
            uint32_t l = 0, f = 0;
            for (const auto *lst : {&pl[r], &mi[r]})
                for (uint32_t x : *lst) (x >= b0 && x < b1 ? l : f) += 1;
            nloc[r - b0] = l;
            nfar[r - b0] = f;
        }
        std::stable_sort(rows.begin(), rows.end(), [&](uint32_t x, uint32_t y) {
            return nfar[x] != nfar[y] ? nfar[x] < nfar[y] : nloc[x] < nloc[y];
        });
        for (uint32_t p = 0; p < b1 - b0; ++p) {
            const uint32_t lr = rows[p], r = b0 + lr;
            pos[b0 + p] = lr;
            off[b0 + p] = (uint32_t)ent.size();
            uint32_t c[4] = {0, 0, 0, 0};
            std::vector<uint32_t> loc;
            for (int part = 0; part < 4; ++part) {
                const std::vector<uint32_t> &lst = (part & 1) ? mi[r] : pl[r];
                const bool local = part < 2;
                for (uint32_t x : lst) {
                    const bool in = x >= b0 && x < b1;
                    if (in != local) continue;
                    if (local) loc.push_back(x - b0);
                    else ent.push_back(x);
                    ++c[part];
                }
                // local entries: 16 bits each, two per word, in 16-byte
                // groups; far entries: one word each, from the next group
                // boundary; padding (never read) points at row 0 / row b0
                if (part == 1) {
                    while (loc.size() % 8) loc.push_back(0u);
                    for (size_t k = 0; k < loc.size(); k += 2) ent.push_back(loc[k] | (loc[k + 1] << 16));
                }
                if (part == 3)
                    while (ent.size() % 4) ent.push_back(b0);
            }
            for (uint32_t k : c) ok = ok && k <= 255;
            // the kernel holds a row's entries in registers: at most 24
            // local (16-bit row indices) and 12 far ones
            const uint32_t nl = c[0] + c[1], nf = c[2] + c[3];
            ok = ok && nl <= 24 && nf <= 12 && b1 - b0 <= 65536;
            cnt[b0 + p] = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
        }
    }
    off[up.dim] = (uint32_t)ent.size();
    T.ft_bits = bits;
    if (!ok) return HPHI_OK;
    ent.resize(ent.size() + 8, 0u);   // the far loop may read one group past a row's list
    HPHI_TRY(upload(T.ft_blk, blk.data(), sizeof(uint32_t) * blk.size()));
    HPHI_TRY(upload(T.ft_pos, pos.data(), sizeof(uint32_t) * pos.size()));
    HPHI_TRY(upload(T.ft_off, off.data(), sizeof(uint32_t) * off.size()));
    HPHI_TRY(upload(T.ft_cnt, cnt.data(), sizeof(uint32_t) * cnt.size()));
    HPHI_TRY(upload(T.ft_ent, ent.data(), sizeof(uint32_t) * ent.size()));
    T.ft_nb = (int)nb;
    T.ft_max_rows = (int)max_rows(blk);
    T.ft_ok = true;
    return HPHI_OK;
}

static int build_hub_fast(hphi_ham *h)
{
    const hphi_basis *b = h->basis;
    const Species &up = b->sp[0], &dn = b->sp[1];
    std::vector<std::vector<uint32_t>> pl, mi;
    // down species: sliced ELL of uint16 columns, plus part then minus part
    split_lists(dn, h->hops_split, pl, mi);
    const int64_t nchunk = (dn.dim + kSellChunk - 1) / kSellChunk;
    std::vector<uint32_t> base(nchunk + 1, 0), wp(nchunk, 0), wm(nchunk, 0);
    for (int64_t j = 0; j < nchunk; ++j) {
        for (int64_t c = j * kSellChunk; c < std::min(dn.dim, (j + 1) * kSellChunk); ++c) {
            wp[j] = std::max<uint32_t>(wp[j], (uint32_t)pl[c].size());
            wm[j] = std::max<uint32_t>(wm[j], (uint32_t)mi[c].size());
        }
        base[j + 1] = base[j] + (wp[j] + wm[j]) * kSellChunk;
    }
    std::vector<uint16_t> ent(std::max<uint32_t>(1, base[nchunk]), (uint16_t)dn.dim);
    for (int64_t j = 0; j < nchunk; ++j)
        for (int l = 0; l < kSellChunk; ++l) {
            const int64_t c = j * kSellChunk + l;
            if (c >= dn.dim) continue;
            for (size_t k = 0; k < pl[c].size(); ++k) ent[base[j] + k * kSellChunk + l] = (uint16_t)pl[c][k];
            for (size_t k = 0; k < mi[c].size(); ++k)
                ent[base[j] + (wp[j] + k) * kSellChunk + l] = (uint16_t)mi[c][k];
        }
    HPHI_TRY(upload(h->hub.fs_base, base.data(), sizeof(uint32_t) * base.size()));
    HPHI_TRY(upload(h->hub.fs_wp, wp.data(), sizeof(uint32_t) * wp.size()));
    HPHI_TRY(upload(h->hub.fs_wm, wm.data(), sizeof(uint32_t) * wm.size()));
    HPHI_TRY(upload(h->hub.fs_ent, ent.data(), sizeof(uint16_t) * ent.size()));
    // down species, hop-ordered slots: slot k of a 64-state chunk is one
    // hop for all its states (the 64 targets of a slot mostly lie in one
    // group of consecutive states). Lane-major: the slots of one state are
    // consecutive, padded to a multiple of 8, so a lane reads 8 per 16-byte
    // load. Two slots per 32-bit word: columns in bits 0..14 and 15..29,
    // their fermion signs in bits 31 and 30; unconnected slots hold dim_dn.
    if (dn.dim < 32768) {
        std::vector<uint32_t> fbase(nchunk + 1, 0), fw(nchunk, 0);
        std::vector<uint32_t> fent, fc4, fc8;
        std::vector<std::vector<uint32_t>> slots;   // column | negative << 16
        // pre-scaled words (element size E = 4 or 8): bits 0..16 hold E times
        // the low slot's column with its sign in bit 0, bits 17..30 the high
        // slot's column and bit 31 its sign; columns (and dim_dn, the padding
        // column) must fit 14 bits
        const bool fc = dn.dim <= 16383;
        auto fc_word = [](uint32_t e0, uint32_t e1, uint32_t esz) {
            return esz * (e0 & 0x7FFFu) | ((e0 >> 16) & 1u) | ((e1 & 0x7FFFu) << 17) | ((e1 >> 16) << 31);
        };
        uint32_t wmax = 0;
        for (int64_t j = 0; j < nchunk; ++j) {
            const int64_t c0 = j * kSellChunk, c1 = std::min(dn.dim, c0 + kSellChunk);
            slots.clear();
            for (const hphi_hop &hp : h->hops_split) {
                bool any = false;
                std::vector<uint32_t> col(kSellChunk, (uint32_t)dn.dim);
                for (int64_t c = c0; c < c1; ++c) {
                    const uint64_t st = dn.state_at(c);
                    if (((st >> hp.i) & 1) == ((st >> hp.j) & 1)) continue;
                    const uint64_t t = st ^ ((uint64_t(1) << hp.i) | (uint64_t(1) << hp.j));
                    const int lo = std::min(hp.i, hp.j), hi = std::max(hp.i, hp.j);
                    const uint64_t between =
                        (hi - lo > 1) ? (((uint64_t(1) << hi) - 1) & ~((uint64_t(1) << (lo + 1)) - 1)) : 0;
                    const int fs = (__builtin_popcountll(st & between) & 1) ? -1 : 1;
                    const int se = fs * (hp.t < 0 ? -1 : 1);
                    col[c - c0] = (uint32_t)dn.rank_of(t) | (se < 0 ? 0x10000u : 0u);
                    any = true;
                }
                if (any) slots.push_back(col);
            }
            const uint32_t w8 = (uint32_t)((slots.size() + 7) / 8 * 8);
            fw[j] = w8;
            wmax = std::max(wmax, w8);
            const size_t at = fent.size();
            fent.resize(at + (size_t)w8 / 2 * kSellChunk, 0);
            if (fc) {
                fc4.resize(fent.size(), 0);
                fc8.resize(fent.size(), 0);
            }
            for (int l = 0; l < kSellChunk; ++l)
                for (uint32_t k = 0; k < w8; k += 2) {
                    const uint32_t e0 = k < slots.size() ? slots[k][l] : (uint32_t)dn.dim;
                    const uint32_t e1 = k + 1 < slots.size() ? slots[k + 1][l] : (uint32_t)dn.dim;
                    const size_t at_w = at + (size_t)l * (w8 / 2) + k / 2;
                    fent[at_w] = (e0 & 0x7FFFu) | ((e1 & 0x7FFFu) << 15) | ((e1 >> 16) << 30) | ((e0 >> 16) << 31);
                    if (fc) {
                        fc4[at_w] = fc_word(e0, e1, 4);
                        fc8[at_w] = fc_word(e0, e1, 8);
                    }
                }
            fbase[j + 1] = (uint32_t)fent.size();
        }
        if (fent.empty()) fent.assign(4, (uint32_t)dn.dim | ((uint32_t)dn.dim << 15));
        HPHI_TRY(upload(h->hub.fb_base, fbase.data(), sizeof(uint32_t) * fbase.size()));
        HPHI_TRY(upload(h->hub.fb_w, fw.data(), sizeof(uint32_t) * fw.size()));
        HPHI_TRY(upload(h->hub.fb_ent, fent.data(), sizeof(uint32_t) * fent.size()));
        h->hub.fb_ok = wmax <= 32;   // the kernel holds up to 32 slots per state
        if (fc && !fc4.empty()) {
            HPHI_TRY(upload(h->hub.fc_ent[0], fc4.data(), sizeof(uint32_t) * fc4.size()));
            HPHI_TRY(upload(h->hub.fc_ent[1], fc8.data(), sizeof(uint32_t) * fc8.size()));
            h->hub.fc_ok = h->hub.fb_ok;
        }
    }
    // up species: CSR, plus entries then minus entries, targets as row
    // element offsets r' * dim_dn
    split_lists(up, h->hops_split, pl, mi);
    std::vector<uint32_t> off(up.dim + 1, 0), mid(up.dim, 0), tgt;
    for (int64_t r = 0; r < up.dim; ++r) {
        off[r] = (uint32_t)tgt.size();
        for (uint32_t x : pl[r]) tgt.push_back((uint32_t)((uint64_t)x * (uint64_t)dn.dim));
        mid[r] = (uint32_t)tgt.size();
        for (uint32_t x : mi[r]) tgt.push_back((uint32_t)((uint64_t)x * (uint64_t)dn.dim));
    }
    off[up.dim] = (uint32_t)tgt.size();
    // the same lists in reverse Cuthill-McKee order of the up rows (the
    // column kernels' processing order with hub_row_order 2): row rr_row[p]
    // is processed at position p, its lists at rr_off[p] .. rr_off[p + 1].
    // Built for up to 2^22 up rows (beyond, index order is used).
    if (up.dim <= (int64_t(1) << 22)) {
        std::vector<std::vector<uint32_t>> adj((size_t)up.dim);
        for (int64_t r = 0; r < up.dim; ++r) {
            adj[r] = pl[r];
            adj[r].insert(adj[r].end(), mi[r].begin(), mi[r].end());
        }
        const std::vector<uint32_t> ord = rcm_order(adj);
        std::vector<uint32_t> roff(up.dim + 1, 0), rmid(up.dim, 0), rent;
        rent.reserve(tgt.size() + 16);
        for (int64_t p = 0; p < up.dim; ++p) {
            const uint32_t r = ord[p];
            roff[p] = (uint32_t)rent.size();
            rent.insert(rent.end(), tgt.begin() + off[r], tgt.begin() + mid[r]);
            rmid[p] = (uint32_t)rent.size();
            rent.insert(rent.end(), tgt.begin() + mid[r], tgt.begin() + off[r + 1]);
        }
        roff[up.dim] = (uint32_t)rent.size();
        rent.resize(rent.size() + 16, 0u);
        HPHI_TRY(upload(h->hub.rr_off, roff.data(), sizeof(uint32_t) * roff.size()));
        HPHI_TRY(upload(h->hub.rr_mid, rmid.data(), sizeof(uint32_t) * rmid.size()));
        HPHI_TRY(upload(h->hub.rr_ent, rent.data(), sizeof(uint32_t) * rent.size()));
        HPHI_TRY(upload(h->hub.rr_row, ord.data(), sizeof(uint32_t) * ord.size()));
    }
    // padding: 16 entries past the last list (row 0 targets, never used)
    tgt.resize(tgt.size() + 16, 0u);
    HPHI_TRY(upload(h->hub.fu_off, off.data(), sizeof(uint32_t) * off.size()));
    HPHI_TRY(upload(h->hub.fu_mid, mid.data(), sizeof(uint32_t) * mid.size()));
    HPHI_TRY(upload(h->hub.fu_ent, tgt.data(), sizeof(uint32_t) * tgt.size()));
    return HPHI_OK;
}

// Two-body tables of one set of values: per-pair records, per-site lists of
// the pairs' other ends with V (the cross weights), and the same-species
// diagonal (V - JH) n_i n_j of each up row and each down state.
struct PairHost {
    std::vector<HubPairDev> rec;
    std::vector<uint32_t> soff;
    std::vector<PairNbrDev> snbr;
    std::vector<double> e[2];
};

static int pair_host_tables(const hphi_basis *b, const hphi_pair_term *pairs, int n_pairs, PairHost &o)
{
    o.rec.assign(n_pairs, HubPairDev{});
    for (int k = 0; k < n_pairs; ++k) {
        const int i = pairs[k].i, j = pairs[k].j;
        if (i < 0 || j < 0 || i >= b->n_sites || j >= b->n_sites || i == j)
            return fail(HPHI_ERR_INVALID_ARG, "pair term %d (%d, %d) invalid for %d sites", k, i, j, b->n_sites);
        const int lo = std::min(i, j), hi = std::max(i, j);
        HubPairDev &q = o.rec[k];
        q.mask = (1u << i) | (1u << j);
        q.between = (hi - lo > 1) ? (((1u << hi) - 1u) & ~((2u << lo) - 1u)) : 0u;
        q.i = i;
        q.j = j;
        q.v = pairs[k].v;
        q.jh = pairs[k].j_hund;
        q.jx = pairs[k].j_ex;
        q.jp = pairs[k].j_pair;
    }
    if (n_pairs == 0) return HPHI_OK;
    if (b->n_sites > 32 || !b->sp[0].d_hi_off32.p || !b->sp[1].d_hi_off32.p)
        return fail(HPHI_ERR_UNSUPPORTED, "two-body terms need at most 32 sites");
    o.soff.assign(b->n_sites + 1, 0);
    for (const HubPairDev &q : o.rec) {
        ++o.soff[q.i + 1];
        ++o.soff[q.j + 1];
    }
    for (int k = 0; k < b->n_sites; ++k) o.soff[k + 1] += o.soff[k];
    o.snbr.assign(o.soff[b->n_sites], PairNbrDev{});
    std::vector<uint32_t> fill(o.soff.begin(), o.soff.end() - 1);
    for (const HubPairDev &q : o.rec) {
        o.snbr[fill[q.i]++] = PairNbrDev{q.j, 0, q.v};
        o.snbr[fill[q.j]++] = PairNbrDev{q.i, 0, q.v};
    }
    for (int sgm = 0; sgm < 2; ++sgm) {
        const Species &sp = b->sp[sgm];
        std::vector<double> &e = o.e[sgm];
        e.assign((size_t)sp.dim, 0.0);
        for (int64_t r = 0; r < sp.dim; ++r) {
            const uint64_t x = sp.state_at(r);
            double s = 0.0;
            for (const HubPairDev &q : o.rec)
                if (((x >> q.i) & 1u) && ((x >> q.j) & 1u)) s += q.v - q.jh;
            e[(size_t)r] = s;
        }
    }
    return HPHI_OK;
}

static int build_hub_pairs(hphi_ham *h, const hphi_pair_term *pairs, int n_pairs)
{
    PairHost o;
    HPHI_TRY(pair_host_tables(h->basis, pairs, n_pairs, o));
    h->pair_terms.assign(pairs, pairs + n_pairs);
    h->hub.n_pairs = n_pairs;
    if (n_pairs == 0) return HPHI_OK;
    HPHI_TRY(upload(h->hub.pairs, o.rec.data(), sizeof(HubPairDev) * o.rec.size()));
    HPHI_TRY(upload(h->hub.pair_site_off, o.soff.data(), sizeof(uint32_t) * o.soff.size()));
    HPHI_TRY(upload(h->hub.pair_site_nbr, o.snbr.data(), sizeof(PairNbrDev) * o.snbr.size()));
    HPHI_TRY(upload(h->hub.pair_eup, o.e[0].data(), sizeof(double) * o.e[0].size()));
    HPHI_TRY(upload(h->hub.pair_edn, o.e[1].data(), sizeof(double) * o.e[1].size()));
    return HPHI_OK;
}

// Groups the frames of one kind into slots of equal values: slot_of[f],
// and the values of each slot (first frame with them) appended to vals.
static int frame_slots(int F, size_t width, const std::function<double(int, size_t)> &at, std::vector<int> &slot_of,
                       std::vector<double> &vals)
{
    std::map<std::vector<double>, int> seen;
    slot_of.assign(F, 0);
    vals.clear();
    std::vector<double> row(width);
    for (int f = 0; f < F; ++f) {
        for (size_t c = 0; c < width; ++c) {
            row[c] = at(f, c);
            if (!std::isfinite(row[c])) return fail(HPHI_ERR_INVALID_ARG, "frame %d: value %zu is not finite", f, c);
        }
        auto it = seen.find(row);
        if (it == seen.end()) {
            it = seen.emplace(row, (int)seen.size()).first;
            vals.insert(vals.end(), row.begin(), row.end());
        }
        slot_of[f] = it->second;
    }
    return HPHI_OK;
}

// Builds a Hubbard Hamiltonian; with frames, the amplitudes of frame 0 are
// in force and the other frames' tables are kept on the device.
static int make_hubbard(hphi_basis *b, const hphi_hop *hops, int n_hops, const double *u_site,
                        const hphi_pair_term *pairs, int n_pairs, const hphi_hub_frames *fr, hphi_ham **out)
{
    if (!b || !out || (n_hops > 0 && !hops) || !u_site || (n_pairs > 0 && !pairs))
        return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (b->kind != 1) return fail(HPHI_ERR_INVALID_ARG, "Hubbard Hamiltonian needs a Hubbard basis");
    if (n_hops < 0 || n_hops > 4096) return fail(HPHI_ERR_INVALID_ARG, "n_hops %d outside [0, 4096]", n_hops);
    if (n_pairs < 0 || n_pairs > kMaxPairTerms)
        return fail(HPHI_ERR_INVALID_ARG, "n_pairs %d outside [0, %d]", n_pairs, kMaxPairTerms);
    if (fr) {
        if (fr->n_frames < 1 || fr->n_frames > kMaxFrames)
            return fail(HPHI_ERR_INVALID_ARG, "n_frames %d outside [1, %d]", fr->n_frames, kMaxFrames);
        if (!fr->hop_t && !fr->hop_t_im && !fr->u_site && !fr->pair_v)
            return fail(HPHI_ERR_INVALID_ARG, "frames without hop_t, hop_t_im, u_site or pair_v");
        if ((fr->hop_t || fr->hop_t_im) && n_hops == 0)
            return fail(HPHI_ERR_INVALID_ARG, "hop_t / hop_t_im frames without hops");
        if (fr->pair_v && n_pairs == 0) return fail(HPHI_ERR_INVALID_ARG, "pair_v frames without pair terms");
    }
    const int F = fr ? fr->n_frames : 1;
    const int ns = b->n_sites;
    DeviceGuard g(b->ctx->device);
    std::unique_ptr<hphi_ham> h(new hphi_ham);
    h->basis = b;
    h->kind = 1;
    for (int k = 0; k < n_hops; ++k) {
        const int i = hops[k].i, j = hops[k].j;
        if (i < 0 || j < 0 || i >= ns || j >= ns || i == j)
            return fail(HPHI_ERR_INVALID_ARG, "hop %d (%d, %d) invalid for %d sites", k, i, j, ns);
    }
    // amplitudes by frame, grouped into slots per kind
    std::vector<int> hop_slot, u_slot, pair_slot;
    std::vector<double> hop_v, u_v, pair_v;
    // hop values of a slot: n_hops real parts, then n_hops imaginary parts
    HPHI_TRY(frame_slots(F, 2 * (size_t)n_hops,
                         [&](int f, size_t c) {
                             if (c < (size_t)n_hops)
                                 return fr && fr->hop_t ? fr->hop_t[(size_t)f * n_hops + c] : hops[c].t;
                             return fr && fr->hop_t_im ? fr->hop_t_im[(size_t)f * n_hops + (c - n_hops)] : 0.0;
                         },
                         hop_slot, hop_v));
    HPHI_TRY(frame_slots(F, (size_t)ns,
                         [&](int f, size_t i) { return fr && fr->u_site ? fr->u_site[(size_t)f * ns + i] : u_site[i]; },
                         u_slot, u_v));
    HPHI_TRY(frame_slots(F, (size_t)n_pairs * 4,
                         [&](int f, size_t c) {
                             if (fr && fr->pair_v) return fr->pair_v[(size_t)f * n_pairs * 4 + c];
                             const hphi_pair_term &q = pairs[c / 4];
                             const double x[4] = {q.v, q.j_hund, q.j_ex, q.j_pair};
                             return x[c % 4];
                         },
                         pair_slot, pair_v));
    const int nhs = n_hops > 0 ? (int)(hop_v.size() / (2 * (size_t)n_hops)) : 1;
    const int nus = (int)(u_v.size() / ns);
    const int nps = n_pairs > 0 ? (int)(pair_v.size() / (4 * (size_t)n_pairs)) : 1;
    auto hop_at = [&](int slot, int k) { return hop_v[(size_t)slot * 2 * n_hops + k]; };
    auto hop_im = [&](int slot, int k) { return hop_v[(size_t)slot * 2 * n_hops + n_hops + k]; };
    bool cplx = false;
    for (int s = 0; s < nhs; ++s)
        for (int k = 0; k < n_hops; ++k)
            if (hop_im(s, k) != 0.0) cplx = true;
    // value classes: matrix elements equal in every slot share one. A row
    // whose state holds site i of hop k takes -t_k, one that holds site j
    // takes -conj(t_k): one class for real transfers, two otherwise.
    std::map<std::vector<double>, int> classes;
    std::vector<int> cls_i(n_hops), cls_j(n_hops);
    std::vector<std::vector<double>> cls_val;   // per class: (re, im) per slot
    auto class_of = [&](const std::vector<double> &key, int &out) -> int {
        auto it = classes.find(key);
        if (it == classes.end()) {
            const int c = (int)classes.size();
            if (c >= (int)kZeroClass) return fail(HPHI_ERR_INVALID_ARG, "more than 127 distinct transfer values");
            it = classes.emplace(key, c).first;
            cls_val.push_back(key);
        }
        out = it->second;
        return HPHI_OK;
    };
    for (int k = 0; k < n_hops; ++k) {
        std::vector<double> ki(2 * (size_t)nhs), kj(2 * (size_t)nhs);
        for (int s = 0; s < nhs; ++s) {
            ki[2 * s] = kj[2 * s] = -hop_at(s, k);
            ki[2 * s + 1] = -hop_im(s, k);
            kj[2 * s + 1] = hop_im(s, k);
        }
        HPHI_TRY(class_of(ki, cls_i[k]));
        if (cplx) HPHI_TRY(class_of(kj, cls_j[k]));
        else cls_j[k] = cls_i[k];
    }
    // per slot: 128 real parts, then 128 imaginary parts
    std::vector<double> coef((size_t)nhs * 256, 0.0);
    for (int s = 0; s < nhs; ++s)
        for (size_t c = 0; c < cls_val.size(); ++c) {
            coef[(size_t)s * 256 + c] = cls_val[c][2 * s];
            coef[(size_t)s * 256 + 128 + c] = cls_val[c][2 * s + 1];
        }
    h->hub.n_coef = (int)classes.size();
    h->hub.cplx = cplx;
    // uniform magnitude: t_k = sg_k tau(slot) in every slot, one sign per hop
    bool uni = n_hops > 0 && !cplx && b->sp[1].dim < 65535 &&
               (unsigned __int128)b->sp[0].dim * (unsigned __int128)b->sp[1].dim * 2 < ((unsigned __int128)1 << 32);
    std::vector<double> tau(nhs, 0.0);
    std::vector<double> sg(n_hops, 1.0);
    int ref = -1;
    for (int s = 0; uni && s < nhs && ref < 0; ++s)
        if (hop_at(s, 0) != 0.0) ref = s;
    if (ref < 0) uni = false;
    if (uni) {
        const double s0 = hop_at(ref, 0) < 0.0 ? -1.0 : 1.0;
        for (int s = 0; s < nhs; ++s) tau[s] = s0 * hop_at(s, 0);
        for (int k = 0; k < n_hops && uni; ++k) {
            const double r = hop_at(ref, k);
            if (r == tau[ref]) sg[k] = 1.0;
            else if (r == -tau[ref]) sg[k] = -1.0;
            else uni = false;
        }
        for (int s = 0; s < nhs && uni; ++s)
            for (int k = 0; k < n_hops && uni; ++k)
                if (hop_at(s, k) != sg[k] * tau[s]) uni = false;
    }
    h->hops.assign(hops, hops + n_hops);
    h->hops_split = h->hops;
    for (int k = 0; k < n_hops; ++k) {
        h->hops[k].t = hop_at(hop_slot[0], k);
        if (uni) h->hops_split[k].t = sg[k] * std::fabs(tau[ref]);
    }
    HPHI_TRY(upload(h->hub.coef, coef.data() + (size_t)hop_slot[0] * 256, sizeof(double) * 128));
    if (cplx) HPHI_TRY(upload(h->hub.coef_im, coef.data() + (size_t)hop_slot[0] * 256 + 128, sizeof(double) * 128));
    const double *u0v = u_v.data() + (size_t)u_slot[0] * ns;
    h->u_site.assign(u0v, u0v + ns);
    HPHI_TRY(upload(h->hub.u_site, u0v, sizeof(double) * ns));
    h->hub.uniform_u = true;
    for (int s = 0; s < nus; ++s)
        for (int i = 1; i < ns; ++i)
            if (u_v[(size_t)s * ns + i] != u_v[(size_t)s * ns]) h->hub.uniform_u = false;
    h->hub.u0 = u0v[0];
    for (int sgm = 0; sgm < 2; ++sgm)
        HPHI_TRY(build_hub_species(b->sp[sgm], h->hops, cls_i, cls_j, h->hub.off[sgm], h->hub.nbr[sgm],
                                   h->hub.max_deg[sgm], h->hub.sell_base[sgm], h->hub.sell_width[sgm],
                                   h->hub.sell[sgm]));
    // uniform-magnitude transfers: the sign-split fast path
    h->hub.uniform_t = uni;
    if (uni) {
        h->hub.t0 = tau[hop_slot[0]];
        HPHI_TRY(build_hub_fast(h.get()));
        HPHI_TRY(build_hub_tile(h.get(), h->sched_cfg.hub_tile_bits));
        // the block-tile T_up kernel where its tables could be built
        if (h->hub.ft_ok) h->sched_cfg.hub_sweep = 7;
    }
    auto pair_terms_of = [&](int slot) {
        std::vector<hphi_pair_term> q(pairs, pairs + n_pairs);
        for (int p = 0; p < n_pairs; ++p) {
            const double *x = pair_v.data() + ((size_t)slot * n_pairs + p) * 4;
            q[p].v = x[0];
            q[p].j_hund = x[1];
            q[p].j_ex = x[2];
            q[p].j_pair = x[3];
        }
        return q;
    };
    {
        const std::vector<hphi_pair_term> q0 = pair_terms_of(pair_slot[0]);
        HPHI_TRY(build_hub_pairs(h.get(), q0.data(), n_pairs));
    }
    if (fr) {
        std::unique_ptr<HubFrames> T(new HubFrames);
        T->n = F;
        T->hop_slot = hop_slot;
        T->u_slot = u_slot;
        T->pair_slot = pair_slot;
        T->cur_hop = hop_slot[0];
        T->cur_u = u_slot[0];
        T->cur_pair = pair_slot[0];
        T->hop_t = hop_v;
        T->tau = tau;
        T->u_site = u_v;
        T->pair_v = pair_v;
        HPHI_TRY(upload(T->coef, coef.data(), sizeof(double) * coef.size()));
        HPHI_TRY(upload(T->u, u_v.data(), sizeof(double) * u_v.size()));
        if (n_pairs > 0) {
            std::vector<HubPairDev> rec;
            std::vector<PairNbrDev> nbr;
            std::vector<double> eup, edn;
            for (int s = 0; s < nps; ++s) {
                const std::vector<hphi_pair_term> q = pair_terms_of(s);
                PairHost o;
                HPHI_TRY(pair_host_tables(b, q.data(), n_pairs, o));
                rec.insert(rec.end(), o.rec.begin(), o.rec.end());
                nbr.insert(nbr.end(), o.snbr.begin(), o.snbr.end());
                eup.insert(eup.end(), o.e[0].begin(), o.e[0].end());
                edn.insert(edn.end(), o.e[1].begin(), o.e[1].end());
                T->nbr_n = o.snbr.size();
            }
            HPHI_TRY(upload(T->pairs, rec.data(), sizeof(HubPairDev) * rec.size()));
            HPHI_TRY(upload(T->nbr, nbr.data(), sizeof(PairNbrDev) * nbr.size()));
            HPHI_TRY(upload(T->eup, eup.data(), sizeof(double) * eup.size()));
            HPHI_TRY(upload(T->edn, edn.data(), sizeof(double) * edn.size()));
        }
        h->td = std::move(T);
    }
    HPHI_TRY(ensure_reduce(h.get()));
    *out = h.release();
    return HPHI_OK;
}

int hphi_ham_hubbard(hphi_basis *b, const hphi_hop *hops, int n_hops, const double *u_site, hphi_ham **out)
{
    return make_hubbard(b, hops, n_hops, u_site, nullptr, 0, nullptr, out);
}

int hphi_ham_hubbard_ext(hphi_basis *b, const hphi_hop *hops, int n_hops, const double *u_site,
                         const hphi_pair_term *pairs, int n_pairs, hphi_ham **out)
{
    return make_hubbard(b, hops, n_hops, u_site, pairs, n_pairs, nullptr, out);
}

int hphi_ham_hubbard_td(hphi_basis *b, const hphi_hop *hops, int n_hops, const double *u_site,
                        const hphi_pair_term *pairs, int n_pairs, const hphi_hub_frames *frames, hphi_ham **out)
{
    if (!frames) return fail(HPHI_ERR_INVALID_ARG, "null frames");
    return make_hubbard(b, hops, n_hops, u_site, pairs, n_pairs, frames, out);
}

extern "C++" {
namespace hphi {

// Puts frame k's slots in force: copies over the live tables on stream st
// (ordered after earlier work on st) and sets the launch-time scalars.
int ham_apply_frame(hphi_ham *h, int k, hipStream_t st)
{
    HubFrames &T = *h->td;
    const hphi_basis *b = h->basis;
    const int ns = b->n_sites, nh = (int)h->hops.size(), np = h->hub.n_pairs;
    const int hs = T.hop_slot[k], us = T.u_slot[k], ps = T.pair_slot[k];
    if (hs != T.cur_hop) {
        HPHI_HIP(hipMemcpyAsync(h->hub.coef.p, T.coef.as<double>() + (size_t)hs * 256, sizeof(double) * 128,
                                hipMemcpyDeviceToDevice, st));
        if (h->hub.cplx)
            HPHI_HIP(hipMemcpyAsync(h->hub.coef_im.p, T.coef.as<double>() + (size_t)hs * 256 + 128,
                                    sizeof(double) * 128, hipMemcpyDeviceToDevice, st));
        if (h->hub.uniform_t) h->hub.t0 = T.tau[hs];
        for (int q = 0; q < nh; ++q) h->hops[q].t = T.hop_t[(size_t)hs * 2 * nh + q];
        T.cur_hop = hs;
    }
    if (us != T.cur_u) {
        HPHI_HIP(hipMemcpyAsync(h->hub.u_site.p, T.u.as<double>() + (size_t)us * ns, sizeof(double) * ns,
                                hipMemcpyDeviceToDevice, st));
        h->u_site.assign(T.u_site.begin() + (size_t)us * ns, T.u_site.begin() + (size_t)(us + 1) * ns);
        h->hub.u0 = h->u_site[0];
        T.cur_u = us;
    }
    if (np > 0 && ps != T.cur_pair) {
        const int64_t dup = b->sp[0].dim, ddn = b->sp[1].dim;
        HPHI_HIP(hipMemcpyAsync(h->hub.pairs.p, T.pairs.as<HubPairDev>() + (size_t)ps * np, sizeof(HubPairDev) * np,
                                hipMemcpyDeviceToDevice, st));
        HPHI_HIP(hipMemcpyAsync(h->hub.pair_site_nbr.p, T.nbr.as<PairNbrDev>() + (size_t)ps * T.nbr_n,
                                sizeof(PairNbrDev) * T.nbr_n, hipMemcpyDeviceToDevice, st));
        HPHI_HIP(hipMemcpyAsync(h->hub.pair_eup.p, T.eup.as<double>() + (size_t)ps * dup, sizeof(double) * dup,
                                hipMemcpyDeviceToDevice, st));
        HPHI_HIP(hipMemcpyAsync(h->hub.pair_edn.p, T.edn.as<double>() + (size_t)ps * ddn, sizeof(double) * ddn,
                                hipMemcpyDeviceToDevice, st));
        for (int p = 0; p < np; ++p) {
            const double *x = T.pair_v.data() + ((size_t)ps * np + p) * 4;
            h->pair_terms[p].v = x[0];
            h->pair_terms[p].j_hund = x[1];
            h->pair_terms[p].j_ex = x[2];
            h->pair_terms[p].j_pair = x[3];
        }
        T.cur_pair = ps;
    }
    T.cur = k;
    return HPHI_OK;
}

} // namespace hphi
} // extern "C++"

int hphi_ham_set_frame(hphi_ham *h, int frame, void *stream)
{
    if (!h) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (!h->td) return fail(HPHI_ERR_INVALID_ARG, "the Hamiltonian has no frames");
    if (frame < 0 || frame >= h->td->n)
        return fail(HPHI_ERR_INVALID_ARG, "frame %d outside [0, %d)", frame, h->td->n);
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    HPHI_USE_HAM(h, st);
    return ham_apply_frame(h, frame, st);
}

int hphi_ham_frames(const hphi_ham *h, int *n_frames, int *current)
{
    if (!h || !n_frames || !current) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    *n_frames = h->td ? h->td->n : 0;
    *current = h->td ? h->td->cur : 0;
    return HPHI_OK;
}

void hphi_ham_free(hphi_ham *h) { delete h; }

int hphi_ham_set_schedule(hphi_ham *h, const hphi_schedule *s)
{
    if (!h || !s) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    hphi_schedule n = h->sched_cfg;
    if (s->hub_slab_cols) {
        if (s->hub_slab_cols != 8 && s->hub_slab_cols != 16 && s->hub_slab_cols != 32 && s->hub_slab_cols != 64 &&
            s->hub_slab_cols != 128)
            return fail(HPHI_ERR_INVALID_ARG, "hub_slab_cols %d", s->hub_slab_cols);
        n.hub_slab_cols = s->hub_slab_cols;
    }
    if (s->hub_groups) {
        if (s->hub_groups < 1 || s->hub_groups > 1024) return fail(HPHI_ERR_INVALID_ARG, "hub_groups %d", s->hub_groups);
        n.hub_groups = s->hub_groups;
    }
    if (s->hub_item_rows) {
        if (s->hub_item_rows < 8 || s->hub_item_rows > 128)
            return fail(HPHI_ERR_INVALID_ARG, "hub_item_rows %d", s->hub_item_rows);
        n.hub_item_rows = s->hub_item_rows;
    }
    if (s->hub_row_cols) {
        if (s->hub_row_cols < 1 || s->hub_row_cols > 6)
            return fail(HPHI_ERR_INVALID_ARG, "hub_row_cols %d", s->hub_row_cols);
        n.hub_row_cols = s->hub_row_cols;
    }
    if (s->spin_per_cu) {
        if (s->spin_per_cu < 1 || s->spin_per_cu > 16) return fail(HPHI_ERR_INVALID_ARG, "spin_per_cu %d", s->spin_per_cu);
        n.spin_per_cu = s->spin_per_cu;
    }
    if (s->spin_implicit) {
        if (s->spin_implicit != 1 && s->spin_implicit != -1)
            return fail(HPHI_ERR_INVALID_ARG, "spin_implicit %d", s->spin_implicit);
        n.spin_implicit = s->spin_implicit == 1 ? 1 : 0;
    }
    if (s->hub_sweep) {
        if (s->hub_sweep != 1 && s->hub_sweep != 3 && s->hub_sweep != 5 && s->hub_sweep != 7)
            return fail(HPHI_ERR_INVALID_ARG, "hub_sweep %d (1, 3, 5 or 7)", s->hub_sweep);
        n.hub_sweep = s->hub_sweep;
    }
    if (s->hub_row_order) {
        if (s->hub_row_order != 1 && s->hub_row_order != 2)
            return fail(HPHI_ERR_INVALID_ARG, "hub_row_order %d", s->hub_row_order);
        n.hub_row_order = s->hub_row_order;
    }
    if (s->spin_tables) {
        if (s->spin_tables != -1 && (s->spin_tables < 1 || s->spin_tables > 3))
            return fail(HPHI_ERR_INVALID_ARG, "spin_tables %d", s->spin_tables);
        n.spin_tables = s->spin_tables == -1 ? 0 : s->spin_tables;
    }
    if (s->spin_split) {
        if (s->spin_split != -1 && (s->spin_split < 1 || s->spin_split > 3))
            return fail(HPHI_ERR_INVALID_ARG, "spin_split %d", s->spin_split);
        n.spin_split = s->spin_split;
    }
    if (s->spin_blk_lo) {
        if (s->spin_blk_lo != -1 && (s->spin_blk_lo < 1 || s->spin_blk_lo > 24))
            return fail(HPHI_ERR_INVALID_ARG, "spin_blk_lo %d", s->spin_blk_lo);
        n.spin_blk_lo = s->spin_blk_lo == -1 ? 0 : s->spin_blk_lo;
    }
    if (s->hub_sweep == 7 && h->kind == 1 && !h->hub.ft_ok && !s->hub_tile_bits)
        return fail(HPHI_ERR_UNSUPPORTED, "hub_sweep 7: no tile tables for this Hamiltonian");
    if (s->hub_tile_bits) {
        if (s->hub_tile_bits != -1 && (s->hub_tile_bits < 1 || s->hub_tile_bits > 32))
            return fail(HPHI_ERR_INVALID_ARG, "hub_tile_bits %d", s->hub_tile_bits);
        n.hub_tile_bits = s->hub_tile_bits == -1 ? 0 : s->hub_tile_bits;
        if (h->kind == 1 && h->hub.uniform_t) {
            DeviceGuard g(h->basis->ctx->device);
            HPHI_USE_HAM(h, nullptr);
            HPHI_TRY(build_hub_tile(h, n.hub_tile_bits));
            if (!h->hub.ft_ok && n.hub_sweep == 7) {
                // keep the tables of the schedule in force
                (void)build_hub_tile(h, h->sched_cfg.hub_tile_bits);
                return fail(HPHI_ERR_UNSUPPORTED, "hub_tile_bits %d: blocks do not fit the tile kernel",
                            s->hub_tile_bits);
            }
        }
    }
    h->sched_cfg = n;
    return HPHI_OK;
}

int hphi_ham_get_schedule(const hphi_ham *h, hphi_schedule *s)
{
    if (!h || !s) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    *s = h->sched_cfg;
    return HPHI_OK;
}

int hphi_ham_trace(hphi_ham *h, double *trace_out, void *stream)
{
    if (!h || !trace_out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    HPHI_USE_HAM(h, st);
    HPHI_TRY(launch_trace(h, reduce_of(h), st));
    HPHI_HIP(hipMemcpyAsync(trace_out, h->red_result.p, sizeof(double), hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    return HPHI_OK;
}

int hphi_mult(hphi_ham *h, hphi_dtype dt, const void *v_dev, void *w_dev, int64_t nvec, void *stream)
{
    if (!h || !v_dev || !w_dev) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (nvec < 1 || nvec > 32) return fail(HPHI_ERR_INVALID_ARG, "nvec %lld outside [1, 32]", (long long)nvec);
    if (dt != HPHI_F64 && dt != HPHI_F32 && dt != HPHI_C128 && dt != HPHI_C64)
        return fail(HPHI_ERR_INVALID_ARG, "unknown dtype %d", (int)dt);
    if (nvec * dtype_lanes(dt) > 32) return fail(HPHI_ERR_INVALID_ARG, "more than 32 real lanes per state");
    if (v_dev == w_dev) return fail(HPHI_ERR_INVALID_ARG, "v and w alias");
    DeviceGuard g(h->basis->ctx->device);
    HPHI_USE_HAM(h, stream);
    MultArgs a{};
    a.dtype = dt;
    a.nvec = (int)nvec;
    a.v = v_dev;
    a.w = w_dev;
    a.stream = (hipStream_t)stream;
    a.red = reduce_of(h);
    return launch_mult(h, a);
}

int hphi_tridiag_lowest(const double *alpha, const double *beta, int n, int k, double *eig_out, double *vec)
{
    return tridiag_lowest(alpha, beta, n, k, eig_out, vec);
}

// ---------------------------------------------------------------- Lanczos --

namespace {

// Sequential 256-byte aligned pieces of a caller-provided device buffer.
struct Carve {
    unsigned char *base;
    size_t cap, off = 0;
    Carve(void *b, size_t c) : base(static_cast<unsigned char *>(b)), cap(c) {}
    static size_t up(size_t n) { return (n + 255) & ~size_t(255); }
    void *take(size_t n)
    {
        void *p = base + off;
        off += up(n);
        return off <= cap ? p : nullptr;
    }
    bool ok() const { return off <= cap; }
};

// HPHI_PROGRESS set in the environment: long solves report each
// convergence check on stderr.
static bool progress_enabled()
{
    static const bool on = std::getenv("HPHI_PROGRESS") != nullptr;
    return on;
}

struct LanczosRun {
    hphi_ham *h;
    int dt;
    int psi_dt = -1;   // type of the Ritz-vector accumulator (default: dt)
    int64_t dim;
    // complex vectors of a Hermitian H: every vector operation runs on the
    // flat array of 2 x dim reals (dim above counts those; alpha and beta
    // stay real), the product on complex vectors of type mult_dt
    bool cview = false;
    int mult_dt = -1;
    // the product does not take the fused dots (complex view, or the split
    // spin product): <q_k, w> and <w, w> in a pass of their own
    bool sep_dots = false;
    // Hubbard: the vectors may be stored with rows padded to whole cache
    // lines (pitch ld >= cols = dim_dn, padding zero); nstore elements each
    int64_t cols = 0, ld = 0, nstore = 0;
    hipStream_t st;
    void *q[3] = {nullptr, nullptr, nullptr};
    DevMem own_q[3];
    DevMem lz_mem, ab;   // LzDev; alpha[max_iter + 1] then beta[max_iter + 2]
    LzDev *lz = nullptr;
    double *alpha = nullptr, *beta = nullptr;
    int cur = 0, prev = 2, wbuf = 1;
    bool timing = false;
    // the update w <- w - alpha s q_k, beta = |w| runs inside the next
    // product's rows kernel (Hubbard, one real vector); the last one after
    // the loop
    bool fused = false;
    std::vector<hipEvent_t> ev;   // pairs around each H*v
    std::vector<hipEvent_t> evm;  // Hubbard: between the rows and the column kernel of each H*v

    ~LanczosRun()
    {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        for (hipEvent_t e : evm) (void)hipEventDestroy(e);
    }

    int mark()
    {
        hipEvent_t e;
        HPHI_HIP(hipEventCreate(&e));
        ev.push_back(e);
        HPHI_HIP(hipEventRecord(e, st));
        return HPHI_OK;
    }

    // total H*v time; with the mid events also the time of the second
    // (column) kernel alone
    int timed(double *seconds, int *calls, double *second_kernel)
    {
        double tot = 0.0, k2 = 0.0;
        for (size_t i = 0; i + 1 < ev.size(); i += 2) {
            float ms = 0.f;
            HPHI_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            tot += ms;
            if (evm.size() == ev.size() / 2) {
                float m2 = 0.f;
                HPHI_HIP(hipEventElapsedTime(&m2, evm[i / 2], ev[i + 1]));
                k2 += m2;
            }
        }
        *seconds = tot * 1e-3;
        *calls = (int)(ev.size() / 2);
        *second_kernel = k2 * 1e-3;
        return HPHI_OK;
    }

    // Device buffers: allocated here, or carved from `ws` (caller-provided
    // workspace, 256-byte aligned pieces; see lanczos_ws_bytes) and zeroed
    // by a kernel.
    int setup(int max_iter, Carve *ws = nullptr)
    {
        fused = !cview && h->kind == 1 && (dt == HPHI_F64 || dt == HPHI_F32) && hub_rows_fused_ok(h, 1);
        sep_dots = cview || (h->kind == 0 && spin_split_mode(h, !spin_stored_path(h)) != 0);
        cols = ld = dim;
        if (h->kind == 1 && !cview) {
            cols = h->basis->sp[1].dim;
            // padded rows only with allocated buffers (the static scratch
            // path keeps the caller's layout and its size formula)
            ld = (fused && !ws) ? hub_lanczos_pitch(h, dt) : cols;
        }
        nstore = dim / cols * ld;
        const size_t bytes = (size_t)nstore * dtype_size(dt);
        const size_t ab_bytes = sizeof(double) * (2 * (size_t)max_iter + 4);
        if (ws) {
            for (auto &p : q) p = ws->take(bytes);
            lz = static_cast<LzDev *>(ws->take(sizeof(LzDev)));
            alpha = static_cast<double *>(ws->take(ab_bytes));
            if (!ws->ok()) return fail(HPHI_ERR_INVALID_ARG, "Lanczos workspace too small");
            HPHI_TRY(launch_zero(lz, sizeof(LzDev), st));
            HPHI_TRY(launch_zero(alpha, ab_bytes, st));
        } else {
            for (int i = 0; i < 3; ++i) {
                HPHI_TRY(own_q[i].alloc(bytes));
                q[i] = own_q[i].p;
                // the padding stays zero: the kernels write whole rows only
                if (ld != cols) HPHI_HIP(hipMemsetAsync(q[i], 0, bytes, st));
            }
            HPHI_TRY(lz_mem.alloc(sizeof(LzDev)));
            HPHI_HIP(hipMemsetAsync(lz_mem.p, 0, sizeof(LzDev), st));
            lz = lz_mem.as<LzDev>();
            HPHI_TRY(ab.alloc(ab_bytes));
            HPHI_HIP(hipMemsetAsync(ab.p, 0, ab.bytes, st));
            alpha = ab.as<double>();
        }
        beta = alpha + max_iter + 1;
        return HPHI_OK;
    }

    int start(const hphi_lanczos_opts *o)
    {
        cur = 0; wbuf = 1; prev = 2;
        const size_t es = dtype_size(dt);
        if (o->v0_dev) {
            if (ld == cols)
                HPHI_HIP(hipMemcpyAsync(q[0], o->v0_dev, (size_t)dim * es, hipMemcpyDeviceToDevice, st));
            else
                HPHI_HIP(hipMemcpy2DAsync(q[0], (size_t)ld * es, o->v0_dev, (size_t)cols * es, (size_t)cols * es,
                                          (size_t)(dim / cols), hipMemcpyDeviceToDevice, st));
        } else if (ld == cols) {
            HPHI_TRY(launch_rng_uniform(dt, q[0], dim, o->seed, st));
        } else {
            HPHI_TRY(launch_rng_uniform_pitched(dt, q[0], dim / cols, cols, ld, o->seed, st));
        }
        Reduce r = reduce_of(h, lz->nrm);
        if (ld == cols) HPHI_TRY(launch_dots(dt, 1, dim, q[0], q[0], r, 1, st));
        else HPHI_TRY(launch_norm2_pitched(dt, q[0], dim, cols, ld, r, st));
        return launch_lz_init(dt, lz, dim, r, st);
    }

    // one Krylov step on the current buffers; first = no v_{k-1} term. In
    // fused mode a non-first step first completes the previous step's
    // update inside the product (q[cur] becomes q_k in place), so the
    // Ritz-vector accumulation of q_k follows the product.
    int step(bool first, const double *svec, void *psi)
    {
        const bool fz = fused && !first;
        const int pdt = psi_dt < 0 ? dt : psi_dt;
        if (psi && !fz) HPHI_TRY(launch_lz_psi_accum(pdt, dt, lz, svec, dim, psi, q[cur], st, cols, ld));
        MultArgs a{};
        a.dtype = cview ? mult_dt : dt;
        a.nvec = 1;
        a.v = q[cur];
        a.w = q[wbuf];
        a.u = first ? nullptr : q[prev];
        a.coef = lz->coef;
        a.dots = sep_dots ? 0 : 1;
        a.dot_raw = 0;
        a.red = reduce_of(h, lz->dot);
        a.stream = st;
        a.ld = (h->kind == 1 && !cview) ? ld : 0;
        if (fz) {
            a.lz = lz;
            a.lz_alpha = alpha;
            a.lz_beta = beta;
            a.lz_q = q[prev];
            a.lz_red = reduce_of(h, lz->nrm);
        }
        if (timing) {
            HPHI_TRY(mark());
            if (h->kind == 1) {
                hipEvent_t e;
                HPHI_HIP(hipEventCreate(&e));
                evm.push_back(e);
                a.ev_mid = e;
            }
        }
        HPHI_TRY(launch_mult(h, a));
        // <q_k, w> and <w, w> over the flat reals (complex vectors: Re of the
        // complex products; for Hermitian H <q_k|H q_k> is real)
        if (sep_dots) HPHI_TRY(launch_dots_xy_yy(dt, 1, dim, q[cur], q[wbuf], reduce_of(h, lz->dot), st));
        if (timing) HPHI_TRY(mark());
        if (psi && fz) HPHI_TRY(launch_lz_psi_accum(pdt, dt, lz, svec, dim, psi, q[cur], st, cols, ld));
        if (!fused)
            HPHI_TRY(launch_lz_update(dt, lz, alpha, beta, nstore, q[wbuf], q[cur], reduce_of(h, lz->nrm), st));
        const int old_prev = prev;
        prev = cur;
        cur = wbuf;
        wbuf = old_prev;
        return HPHI_OK;
    }

    int run(int n_iter, bool graph, const double *svec, void *psi, int check_every, double tol,
            int n_energies, int *converged, std::vector<double> &last_ev, double resid_tol = 0.0)
    {
        int k = 0;
        HPHI_TRY(step(true, svec, psi));
        ++k;
        if (graph && n_iter - k >= 6 && check_every == 0 && !psi) {
            hipGraph_t gph;
            hipGraphExec_t exec;
            HPHI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
            int rc = HPHI_OK;
            for (int t = 0; t < 3 && rc == HPHI_OK; ++t) rc = step(false, nullptr, nullptr);
            hipError_t e = hipStreamEndCapture(st, &gph);
            if (rc != HPHI_OK) return rc;
            if (e != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
            HPHI_HIP(hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0));
            while (n_iter - k >= 3) {
                HPHI_HIP(hipGraphLaunch(exec, st));
                k += 3;
            }
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(gph);
        }
        std::vector<double> ha, hb;
        for (; k < n_iter; ++k) {
            HPHI_TRY(step(false, svec, psi));
            if (check_every > 0 && (k + 1) % check_every == 0) {
                LzDev hl;
                HPHI_HIP(hipMemcpyAsync(&hl, lz, sizeof(LzDev), hipMemcpyDeviceToHost, st));
                HPHI_HIP(hipStreamSynchronize(st));
                const int n = hl.iter;
                if (hl.done || n < n_energies) {
                    if (hl.done) break;
                    continue;
                }
                ha.resize(n);
                hb.resize(n + 1);
                HPHI_HIP(hipMemcpy(ha.data(), alpha, sizeof(double) * n, hipMemcpyDeviceToHost));
                HPHI_HIP(hipMemcpy(hb.data(), beta, sizeof(double) * (n + 1), hipMemcpyDeviceToHost));
                std::vector<double> ev(n_energies);
                HPHI_TRY(tridiag_lowest(ha.data(), hb.data(), n, n_energies, ev.data(), nullptr));
                if (progress_enabled())
                    std::fprintf(stderr, "hphi_lanczos: %d iterations, lowest Ritz value %.15g\n", n, ev[0]);
                bool ok = last_ev.size() == ev.size();
                for (size_t i = 0; ok && i < ev.size(); ++i)
                    ok = std::fabs(ev[i] - last_ev[i]) < tol * std::max(1.0, std::fabs(ev[i]));
                if (ok && resid_tol > 0.0) {
                    // residual estimate of the lowest Ritz pair: beta_n |s_{n-1}|
                    std::vector<double> sv(n);
                    double th = 0.0;
                    HPHI_TRY(tridiag_lowest(ha.data(), hb.data(), n, 1, &th, sv.data()));
                    ok = hb[n] * std::fabs(sv[n - 1]) < resid_tol * std::max(1.0, std::fabs(th));
                }
                last_ev = ev;
                if (ok) {
                    *converged = 1;
                    break;
                }
            }
        }
        // fused mode: the last product's update (not needed by the
        // Ritz-vector pass, which accumulates q_0 .. q_{n-1} only)
        if (fused && !psi)
            HPHI_TRY(launch_lz_update(dt, lz, alpha, beta, nstore, q[cur], q[prev], reduce_of(h, lz->nrm), st));
        return HPHI_OK;
    }
};

} // namespace

// Lowest Ritz value of T_n distinct from the first (ghost copies of the
// first, which plain Lanczos produces once it has converged, are skipped);
// NaN if there is none.
static double second_distinct_ritz(const std::vector<double> &a, const std::vector<double> &b, int n)
{
    const int k = std::min(n, 8);
    if (k < 2) return NAN;
    std::vector<double> ev(k);
    if (tridiag_lowest(a.data(), b.data(), n, k, ev.data(), nullptr) != HPHI_OK) return NAN;
    for (int i = 1; i < k; ++i)
        if (ev[i] - ev[0] > 1e-6 * std::max(1.0, std::fabs(ev[0]))) return ev[i];
    return NAN;
}

// The Lanczos solve behind hphi_lanczos and hphi_lanczos_noalloc. ws: null
// = allocate the device buffers here; otherwise every device buffer is
// carved from ws (no allocation, no graph, no events).
static int lanczos_impl(hphi_ham *h, const hphi_lanczos_opts *o, double *energies, int n_energies,
                        hphi_lanczos_info *info, Carve *ws)
{
    if (!h || !o || (n_energies > 0 && !energies)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (o->max_iter < 1 || o->max_iter > 100000) return fail(HPHI_ERR_INVALID_ARG, "max_iter %d", o->max_iter);
    const bool cst = o->storage == HPHI_C128 || o->storage == HPHI_C64;
    if (o->storage != HPHI_F64 && o->storage != HPHI_F32 && !cst)
        return fail(HPHI_ERR_INVALID_ARG, "Lanczos storage must be F64, F32, C128 or C64");
    if (cst && (o->refine || ws))
        return fail(HPHI_ERR_INVALID_ARG, "complex Lanczos storage: no refinement and no static scratch");
    if (n_energies < 0 || n_energies > o->max_iter) return fail(HPHI_ERR_INVALID_ARG, "n_energies %d", n_energies);
    if (o->check_every < 0) return fail(HPHI_ERR_INVALID_ARG, "check_every < 0");
    if (o->refine != 0 && o->refine != 1) return fail(HPHI_ERR_INVALID_ARG, "refine %d", o->refine);
    if (o->refine_steps > 1000) return fail(HPHI_ERR_INVALID_ARG, "refine_steps %d", o->refine_steps);
    if (o->resid_tol < 0.0 || !std::isfinite(o->resid_tol)) return fail(HPHI_ERR_INVALID_ARG, "resid_tol");
    DeviceGuard g(h->basis->ctx->device);
    HPHI_USE_HAM(h, o->stream);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)o->stream;
    hipStream_t own = nullptr;
    if (o->use_graph && !st) {
        HPHI_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
        st = own;
    }
    struct StreamDrop {
        hipStream_t s;
        ~StreamDrop() { if (s) (void)hipStreamDestroy(s); }
    } drop{own};
    LanczosRun L;
    L.h = h;
    L.dt = cst ? (o->storage == HPHI_C128 ? HPHI_F64 : HPHI_F32) : o->storage;
    L.dim = h->basis->dim * (cst ? 2 : 1);
    L.cview = cst;
    L.mult_dt = o->storage;
    L.st = st;
    L.timing = o->time_kernels != 0 && !o->use_graph;
    HPHI_TRY(L.setup(o->max_iter, ws));
    HPHI_TRY(L.start(o));
    int converged = 0;
    std::vector<double> last_ev;
    HPHI_TRY(L.run(o->max_iter, o->use_graph != 0, nullptr, nullptr, o->check_every, o->tol,
                   std::max(1, n_energies), &converged, last_ev, o->resid_tol));
    LzDev hl;
    HPHI_HIP(hipMemcpyAsync(&hl, L.lz, sizeof(LzDev), hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    const int n = hl.iter;
    std::vector<double> ha(n), hb(n + 1);
    HPHI_HIP(hipMemcpy(ha.data(), L.alpha, sizeof(double) * n, hipMemcpyDeviceToHost));
    HPHI_HIP(hipMemcpy(hb.data(), L.beta, sizeof(double) * (n + 1), hipMemcpyDeviceToHost));
    hb[0] = 0.0;
    if (o->alpha_out) std::memcpy(o->alpha_out, ha.data(), sizeof(double) * n);
    if (o->beta_out) std::memcpy(o->beta_out, hb.data(), sizeof(double) * n);
    const int ne = std::min(n_energies, n);
    if (ne > 0) HPHI_TRY(tridiag_lowest(ha.data(), hb.data(), n, ne, energies, nullptr));
    for (int i = ne; i < n_energies; ++i) energies[i] = NAN;
    double hv_s = 0.0, hv_k2 = 0.0;
    int hv_n = 0;
    if (L.timing) HPHI_TRY(L.timed(&hv_s, &hv_n, &hv_k2));
    L.timing = false;
    double ritz_e0 = NAN, rq_e0 = NAN, resid = NAN, err_est = NAN, polish_e0 = NAN, polish_resid = NAN;
    if ((o->psi_dev || o->refine) && n > 0) {
        // second pass: same start vector and kernels, psi = sum_k s_k v_k;
        // with refine the sum is kept in FP64 whatever the storage type
        std::vector<double> s(n);
        HPHI_TRY(tridiag_lowest(ha.data(), hb.data(), n, 1, &ritz_e0, s.data()));
        DevMem sv_m, psi64_m, hpsi_m;
        double *sv = nullptr;
        void *psi64 = nullptr, *hpsi = nullptr;
        if (ws) {
            sv = static_cast<double *>(ws->take(sizeof(double) * n));
            if (o->refine) {
                psi64 = ws->take((size_t)L.dim * sizeof(double));
                hpsi = ws->take((size_t)L.dim * sizeof(double));
            }
            if (!ws->ok()) return fail(HPHI_ERR_INVALID_ARG, "Lanczos workspace too small");
            HPHI_HIP(hipMemcpyAsync(sv, s.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
        } else {
            HPHI_TRY(upload(sv_m, s.data(), sizeof(double) * n));
            sv = sv_m.as<double>();
            if (o->refine) {
                HPHI_TRY(psi64_m.alloc((size_t)L.dim * sizeof(double)));
                HPHI_TRY(hpsi_m.alloc((size_t)L.dim * sizeof(double)));
                psi64 = psi64_m.p;
                hpsi = hpsi_m.p;
            }
        }
        void *psi = o->psi_dev;
        int pdt = L.dt;
        if (o->refine) {
            psi = psi64;
            pdt = HPHI_F64;
        }
        L.psi_dt = pdt;
        if (ws) HPHI_TRY(launch_zero(psi, (size_t)L.dim * dtype_size(pdt), st));
        else HPHI_HIP(hipMemsetAsync(psi, 0, (size_t)L.dim * dtype_size(pdt), st));
        HPHI_TRY(L.start(o));
        std::vector<double> dummy;
        int cv = 0;
        HPHI_TRY(L.run(n, false, sv, psi, 0, 0.0, 1, &cv, dummy));
        double *res = h->red_result.as<double>();
        HPHI_TRY(launch_dots(pdt, 1, L.dim, psi, psi, reduce_of(h), 1, st));
        HPHI_TRY(launch_scale_lanes(pdt, 1, L.dim, psi, res, 1, st));
        if (o->refine) {
            // rho = <psi|H psi> and eps = |H psi - rho psi| in FP64
            MultArgs a{};
            a.dtype = HPHI_F64;
            a.nvec = 1;
            a.v = psi;
            a.w = hpsi;
            a.stream = st;
            a.red = reduce_of(h);
            HPHI_TRY(launch_mult(h, a));
            HPHI_TRY(launch_dots(HPHI_F64, 1, L.dim, psi, hpsi, reduce_of(h), 0, st));
            HPHI_HIP(hipMemcpyAsync(&rq_e0, res, sizeof(double), hipMemcpyDeviceToHost, st));
            HPHI_HIP(hipStreamSynchronize(st));
            HPHI_TRY(launch_axpy_lanes(HPHI_F64, 1, L.dim, hpsi, psi, nullptr, -rq_e0, st));
            HPHI_TRY(launch_dots(HPHI_F64, 1, L.dim, hpsi, hpsi, reduce_of(h), 1, st));
            double r2 = 0.0;
            HPHI_HIP(hipMemcpyAsync(&r2, res, sizeof(double), hipMemcpyDeviceToHost, st));
            HPHI_HIP(hipStreamSynchronize(st));
            resid = std::sqrt(std::max(0.0, r2));
            const double th2 = second_distinct_ritz(ha, hb, n);
            if (std::isfinite(th2) && th2 > rq_e0) err_est = r2 / (th2 - rq_e0);
            if (n_energies > 0) energies[0] = rq_e0;
            if (o->psi_dev) HPHI_TRY(launch_copy_cast(L.dt, o->psi_dev, HPHI_F64, psi, L.dim, st));
            // FP64 restart from psi: a few Lanczos steps whose Krylov space
            // holds psi, so the lowest Ritz value is at most rho
            const int rs = o->refine_steps == 0 ? 16 : o->refine_steps;
            if (rs > 0) {
                LanczosRun P;
                P.h = h;
                P.dt = HPHI_F64;
                P.dim = L.dim;
                P.st = st;
                HPHI_TRY(P.setup(rs, ws));
                hphi_lanczos_opts po = *o;
                po.v0_dev = psi;
                po.storage = HPHI_F64;
                HPHI_TRY(P.start(&po));
                std::vector<double> dum;
                int cvp = 0;
                HPHI_TRY(P.run(rs, false, nullptr, nullptr, 0, 0.0, 1, &cvp, dum));
                LzDev hp;
                HPHI_HIP(hipMemcpyAsync(&hp, P.lz, sizeof(LzDev), hipMemcpyDeviceToHost, st));
                HPHI_HIP(hipStreamSynchronize(st));
                const int np = hp.iter;
                if (np > 0) {
                    std::vector<double> pa(np), pb(np + 1), ps(np);
                    HPHI_HIP(hipMemcpy(pa.data(), P.alpha, sizeof(double) * np, hipMemcpyDeviceToHost));
                    HPHI_HIP(hipMemcpy(pb.data(), P.beta, sizeof(double) * (np + 1), hipMemcpyDeviceToHost));
                    HPHI_TRY(tridiag_lowest(pa.data(), pb.data(), np, 1, &polish_e0, ps.data()));
                    polish_resid = pb[np] * std::fabs(ps[np - 1]);
                    if (n_energies > 0) energies[0] = polish_e0;
                }
            }
        }
        HPHI_HIP(hipStreamSynchronize(st));
    }
    if (info) {
        info->iterations = n;
        info->converged = converged;
        info->breakdown = hl.breakdown;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        info->hv_seconds = hv_s;
        info->hv_calls = hv_n;
        info->fused_update = L.fused ? 1 : 0;
        info->hv_second_kernel_seconds = hv_k2;
        info->ritz_e0 = o->refine ? ritz_e0 : NAN;
        info->rq_e0 = rq_e0;
        info->residual = resid;
        info->err_est = err_est;
        info->polish_e0 = polish_e0;
        info->polish_resid = polish_resid;
    }
    return HPHI_OK;
}


int hphi_lanczos(hphi_ham *h, const hphi_lanczos_opts *o, double *energies, int n_energies,
                 hphi_lanczos_info *info)
{
    return lanczos_impl(h, o, energies, n_energies, info, nullptr);
}

} // extern "C"

// Device bytes hphi_lanczos_noalloc carves from the static scratch.
static size_t noalloc_bytes(int64_t dim, int storage, int max_iter, int refine, int refine_steps)
{
    const size_t vb = (size_t)dim * (storage == HPHI_F32 ? 4 : 8);
    size_t n = 3 * Carve::up(vb) + Carve::up(sizeof(LzDev)) + Carve::up(sizeof(double) * (2 * (size_t)max_iter + 4)) +
               Carve::up(sizeof(double) * (size_t)max_iter);
    if (refine) {
        const int rs = refine_steps == 0 ? 16 : refine_steps;
        n += 2 * Carve::up((size_t)dim * sizeof(double));
        if (rs > 0)
            n += 3 * Carve::up((size_t)dim * sizeof(double)) + Carve::up(sizeof(LzDev)) +
                 Carve::up(sizeof(double) * (2 * (size_t)rs + 4));
    }
    return n;
}

static_assert(HPHI_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "scratch size in the header");

extern "C" {

int hphi_lanczos_noalloc(hphi_ham *h, const hphi_lanczos_opts *o, double *energies, int n_energies,
                         hphi_lanczos_info *info)
{
    if (!h || !o) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (o->use_graph || o->time_kernels)
        return fail(HPHI_ERR_INVALID_ARG, "hphi_lanczos_noalloc: use_graph and time_kernels are not available");
    if (o->max_iter < 1 || o->max_iter > 100000) return fail(HPHI_ERR_INVALID_ARG, "max_iter %d", o->max_iter);
    if (o->storage != HPHI_F64 && o->storage != HPHI_F32)
        return fail(HPHI_ERR_INVALID_ARG, "Lanczos storage must be F64 or F32");
    const size_t need = noalloc_bytes(h->basis->dim, o->storage, o->max_iter, o->refine, o->refine_steps);
    if (need > kNoAllocScratchBytes)
        return fail(HPHI_ERR_INVALID_ARG,
                    "hphi_lanczos_noalloc: %zu bytes of workspace needed (dim %lld), the static scratch holds %zu",
                    need, (long long)h->basis->dim, kNoAllocScratchBytes);
    const int dev = h->basis->ctx->device;
    DeviceGuard g(dev);
    void *p = nullptr;
    HPHI_TRY(noalloc_scratch_acquire(dev, &p));
    struct Release {
        int d;
        ~Release() { noalloc_scratch_release(d); }
    } rel{dev};
    struct NoAllocMark {
        hphi_ham *h;
        ~NoAllocMark() { h->noalloc_call = false; }
    } mark{h};
    h->noalloc_call = true;
    Carve ws(p, kNoAllocScratchBytes);
    return lanczos_impl(h, o, energies, n_energies, info, &ws);
}

} // extern "C"

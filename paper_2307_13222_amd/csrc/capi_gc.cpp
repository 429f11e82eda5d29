// SpinGC: the full 2^N spin-1/2 space (SpinGC keyword, HPhi update paper
// Sec. 4.1) -- basis, Hamiltonian and the bit-window plans of its H*v.
#include <algorithm>
#include <cmath>
#include <memory>

#include "internal.h"

namespace hphi {

// Windows for one element size: every off-diagonal term's flip mask, less
// the low bits, must lie in one window of at most qmax bits, with qmax set
// by a 64 KB tile. Terms are taken in order of their highest bit and join
// the last window while the union fits; windows are then filled up to qmax
// bits with the lowest free bits (larger tiles, fewer of them).
int gc_plan_build(hphi_ham *h, int pidx)
{
    GcPlan &plan = h->gc_plan[pidx];
    if (plan.built) return HPHI_OK;
    const int n = h->basis->n_sites;
    const int esz = pidx == 0 ? 4 : (pidx == 1 ? 8 : 16);
    const int lowb = std::min(4, n);
    int qmax = 0;
    while (((size_t)1 << (lowb + qmax + 1)) * esz <= (size_t)64 * 1024) ++qmax;
    qmax = std::min(qmax, n - lowb);
    const uint32_t full = n >= 32 ? 0xFFFFFFFFu : ((1u << n) - 1u);
    const uint32_t lowmask = (1u << lowb) - 1u;
    struct T { uint32_t mask; int i, j; double cpar, canti; };
    std::vector<T> terms;
    for (const hphi_xyz_bond &bd : h->xyz)
        if (bd.jx != 0.0 || bd.jy != 0.0)
            terms.push_back({(1u << bd.i) | (1u << bd.j), bd.i, bd.j, 0.25 * (bd.jx - bd.jy), 0.25 * (bd.jx + bd.jy)});
    for (int i = 0; i < n && !h->hx.empty(); ++i)
        if (h->hx[i] != 0.0) terms.push_back({1u << i, i, i, -0.5 * h->hx[i], -0.5 * h->hx[i]});
    std::stable_sort(terms.begin(), terms.end(), [&](const T &x, const T &y) {
        const uint32_t hx_ = x.mask & ~lowmask, hy = y.mask & ~lowmask;
        const int tx = hx_ ? 31 - __builtin_clz(hx_) : -1, ty = hy ? 31 - __builtin_clz(hy) : -1;
        return tx < ty;
    });
    std::vector<uint32_t> wmask;
    std::vector<int> owner(terms.size(), -1);
    for (size_t k = 0; k < terms.size(); ++k) {
        const uint32_t hb = terms[k].mask & ~lowmask;
        if (!hb) continue;   // placed in the first window below
        for (size_t w = 0; w < wmask.size() && owner[k] < 0; ++w)
            if ((wmask[w] & hb) == hb) owner[k] = (int)w;
        if (owner[k] >= 0) continue;
        if (!wmask.empty() && __builtin_popcount(wmask.back() | hb) <= qmax) {
            wmask.back() |= hb;
            owner[k] = (int)wmask.size() - 1;
        } else {
            if (__builtin_popcount(hb) > qmax) return fail(HPHI_ERR_UNSUPPORTED, "SpinGC: a term spans more than a window");
            wmask.push_back(hb);
            owner[k] = (int)wmask.size() - 1;
        }
    }
    if (wmask.empty()) wmask.push_back(0u);
    for (size_t k = 0; k < terms.size(); ++k)
        if (owner[k] < 0) owner[k] = 0;
    for (uint32_t &wm : wmask)
        for (int bit = lowb; bit < n && __builtin_popcount(wm) < qmax; ++bit) wm |= 1u << bit;
    plan.wins.clear();
    std::vector<uint32_t> offw;
    std::vector<GcTermDev> dev;
    for (size_t w = 0; w < wmask.size(); ++w) {
        GcWindow g;
        g.wmask = wmask[w];
        g.q = __builtin_popcount(wmask[w]);
        g.compmask = full & ~wmask[w] & ~lowmask;
        g.offw_first = offw.size();
        int pos[32];
        int nb = 0;
        for (int bit = 0; bit < 32; ++bit)
            if ((wmask[w] >> bit) & 1u) pos[nb++] = bit;
        for (uint32_t k = 0; k < (1u << g.q); ++k) {
            uint32_t x = 0;
            for (int t = 0; t < g.q; ++t)
                if ((k >> t) & 1u) x |= 1u << pos[t];
            offw.push_back(x);
        }
        // local position of a global bit: low bits stay, window bits follow
        auto loc = [&](int bit) -> int {
            if (bit < lowb) return bit;
            for (int t = 0; t < g.q; ++t)
                if (pos[t] == bit) return lowb + t;
            return -1;
        };
        g.term_first = (int)dev.size();
        for (size_t k = 0; k < terms.size(); ++k) {
            if (owner[k] != (int)w) continue;
            const T &t = terms[k];
            GcTermDev d{};
            const int li = loc(t.i), lj = loc(t.j);
            if (li < 0 || lj < 0) return fail(HPHI_ERR_DEVICE, "SpinGC window plan inconsistent");
            d.mloc = (1u << li) | (1u << lj);
            d.pi = (uint32_t)li;
            d.pj = (uint32_t)lj;
            d.cpar = t.cpar;
            d.canti = t.canti;
            dev.push_back(d);
        }
        g.term_count = (int)dev.size() - g.term_first;
        plan.wins.push_back(g);
    }
    plan.lowb = lowb;
    HPHI_TRY(upload(plan.offw, offw.data(), sizeof(uint32_t) * offw.size()));
    if (dev.empty()) dev.push_back(GcTermDev{});
    HPHI_TRY(upload(plan.terms, dev.data(), sizeof(GcTermDev) * dev.size()));
    plan.built = true;
    return HPHI_OK;
}

} // namespace hphi

using namespace hphi;

extern "C" {

int hphi_basis_spin_gc(hphi_ctx *ctx, int n_sites, hphi_basis **out)
{
    if (!ctx || !out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (n_sites < 1 || n_sites > 32) return fail(HPHI_ERR_INVALID_ARG, "n_sites %d outside [1, 32]", n_sites);
    std::unique_ptr<hphi_basis> b(new hphi_basis);
    b->ctx = ctx;
    b->kind = 2;
    b->n_sites = n_sites;
    b->dim = (int64_t)1 << n_sites;
    *out = b.release();
    return HPHI_OK;
}

int hphi_ham_spin_gc(hphi_basis *b, const hphi_xyz_bond *bonds, int n_bonds, const double *hx, const double *hz,
                     hphi_ham **out)
{
    if (!b || !out || (n_bonds > 0 && !bonds)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (b->kind != 2) return fail(HPHI_ERR_INVALID_ARG, "SpinGC Hamiltonian needs a SpinGC basis");
    if (n_bonds < 0 || n_bonds > 4096) return fail(HPHI_ERR_INVALID_ARG, "n_bonds %d outside [0, 4096]", n_bonds);
    DeviceGuard g(b->ctx->device);
    std::unique_ptr<hphi_ham> h(new hphi_ham);
    h->basis = b;
    h->kind = 2;
    std::vector<GcDiagDev> diag;
    for (int k = 0; k < n_bonds; ++k) {
        const int i = bonds[k].i, j = bonds[k].j;
        if (i < 0 || j < 0 || i >= b->n_sites || j >= b->n_sites || i == j)
            return fail(HPHI_ERR_INVALID_ARG, "bond %d (%d, %d) invalid for %d sites", k, i, j, b->n_sites);
        h->xyz.push_back(bonds[k]);
        if (bonds[k].jz != 0.0) diag.push_back(GcDiagDev{(1u << i) | (1u << j), 0u, 0.25 * bonds[k].jz});
    }
    if (hx) h->hx.assign(hx, hx + b->n_sites);
    if (hz) {
        h->hz_gc.assign(hz, hz + b->n_sites);
        h->gc_has_hz = true;
        HPHI_TRY(upload(h->gc_hz, hz, sizeof(double) * b->n_sites));
    }
    h->gc_ndiag = (int)diag.size();
    if (diag.empty()) diag.push_back(GcDiagDev{});
    HPHI_TRY(upload(h->gc_diag, diag.data(), sizeof(GcDiagDev) * diag.size()));
    HPHI_TRY(ham_ensure_reduce(h.get()));
    *out = h.release();
    return HPHI_OK;
}

} // extern "C"

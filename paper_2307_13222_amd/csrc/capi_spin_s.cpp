// Spin-S sector basis and Hamiltonian (keyword 2S, HPhi update paper
// Sec. 4.1, "Remarks on the keyword model").
#include <cmath>
#include <memory>

#include "internal.h"

using namespace hphi;

int64_t SpinSTables::rank_of(uint64_t x) const
{
    const int n_fields = (lo_bits + hi_bits) / bits;
    if (lo_bits + hi_bits < 64 && (x >> (lo_bits + hi_bits)) != 0) return -1;
    int sum = 0;
    for (int l = 0; l < n_fields; ++l) {
        const int d = (int)((x >> (l * bits)) & ((1ull << bits) - 1ull));
        if (d > two_s) return -1;
        sum += d;
    }
    if (sum != msum) return -1;
    return (int64_t)hi_off[x >> lo_bits] + lo_rank[x & ((1ull << lo_bits) - 1ull)];
}

namespace {

int field_bits(int two_s)
{
    int b = 1;
    while ((1 << b) <= two_s) ++b;
    return b;
}

// digit sum of a pattern of n fields, or -1 if a digit exceeds 2S
int digit_sum(uint64_t x, int n, int bits, int two_s)
{
    int s = 0;
    for (int l = 0; l < n; ++l) {
        const int d = (int)((x >> (l * bits)) & ((1ull << bits) - 1ull));
        if (d > two_s) return -1;
        s += d;
    }
    return s;
}

} // namespace

extern "C" {

int hphi_basis_spin_s(hphi_ctx *ctx, int n_sites, int two_s, int two_sz, hphi_basis **out)
{
    if (!ctx || !out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (two_s < 1 || two_s > 7) return fail(HPHI_ERR_INVALID_ARG, "2S = %d outside [1, 7]", two_s);
    const int bits = field_bits(two_s);
    if (n_sites < 1 || n_sites * bits > 40)
        return fail(HPHI_ERR_INVALID_ARG, "%d sites of %d bits outside [1, 40] bits", n_sites, bits);
    const int msum2 = two_sz + n_sites * two_s;
    if (std::abs(two_sz) > n_sites * two_s || (msum2 & 1))
        return fail(HPHI_ERR_INVALID_ARG, "2Sz = %d impossible for %d spins of 2S = %d", two_sz, n_sites, two_s);
    DeviceGuard g(ctx->device);
    std::unique_ptr<hphi_basis> b(new hphi_basis);
    b->ctx = ctx;
    b->kind = 3;
    b->n_sites = n_sites;
    SpinSTables &t = b->ss;
    t.two_s = two_s;
    t.bits = bits;
    t.msum = msum2 / 2;
    const int n_lo = n_sites / 2, n_hi = n_sites - n_lo;
    t.lo_bits = n_lo * bits;
    t.hi_bits = n_hi * bits;
    const uint64_t nl = 1ull << t.lo_bits, nh = 1ull << t.hi_bits;
    // lo patterns: rank among the valid ones of equal digit sum; and the
    // ascending lists per sum for the enumeration below
    t.lo_rank.assign(nl, 0xFFFFFFFFu);
    std::vector<std::vector<uint32_t>> by_sum(n_lo * two_s + 1);
    for (uint64_t l = 0; l < nl; ++l) {
        const int s = digit_sum(l, n_lo, bits, two_s);
        if (s < 0) continue;
        t.lo_rank[l] = (uint32_t)by_sum[s].size();
        by_sum[s].push_back((uint32_t)l);
    }
    t.hi_off.assign(nh + 1, 0);
    uint64_t acc = 0;
    for (uint64_t hh = 0; hh < nh; ++hh) {
        t.hi_off[hh] = acc;
        const int s = digit_sum(hh, n_hi, bits, two_s);
        const int need = t.msum - s;
        if (s >= 0 && need >= 0 && need <= n_lo * two_s) acc += by_sum[need].size();
    }
    t.hi_off[nh] = acc;
    if (acc == 0) return fail(HPHI_ERR_EMPTY_SECTOR, "empty sector");
    if (acc >= (1ull << 32)) return fail(HPHI_ERR_DIM_OVERFLOW, "spin-S sector of %llu states beyond 2^32",
                                         (unsigned long long)acc);
    b->dim = (int64_t)acc;
    t.states.reserve(acc);
    for (uint64_t hh = 0; hh < nh; ++hh) {
        const int s = digit_sum(hh, n_hi, bits, two_s);
        const int need = t.msum - s;
        if (s < 0 || need < 0 || need > n_lo * two_s) continue;
        for (uint32_t l : by_sum[need]) t.states.push_back((hh << t.lo_bits) | l);
    }
    std::vector<uint32_t> h32(t.hi_off.begin(), t.hi_off.end());
    HPHI_TRY(upload(t.d_hi_off32, h32.data(), sizeof(uint32_t) * h32.size()));
    HPHI_TRY(upload(t.d_lo_rank, t.lo_rank.data(), sizeof(uint32_t) * t.lo_rank.size()));
    HPHI_TRY(upload(t.d_states, t.states.data(), sizeof(uint64_t) * t.states.size()));
    *out = b.release();
    return HPHI_OK;
}

int hphi_ham_spin_s(hphi_basis *b, const hphi_spin_bond *bonds, int n_bonds, const double *hz, const double *d_ion,
                    hphi_ham **out)
{
    if (!b || !out || (n_bonds > 0 && !bonds)) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (b->kind != 3) return fail(HPHI_ERR_INVALID_ARG, "spin-S Hamiltonian needs a spin-S basis");
    if (n_bonds < 0 || n_bonds > 4096) return fail(HPHI_ERR_INVALID_ARG, "n_bonds %d outside [0, 4096]", n_bonds);
    DeviceGuard g(b->ctx->device);
    std::unique_ptr<hphi_ham> h(new hphi_ham);
    h->basis = b;
    h->kind = 3;
    struct Dev { int32_t i, j; double jz, jxy2; };
    std::vector<Dev> dev;
    for (int k = 0; k < n_bonds; ++k) {
        const int i = bonds[k].i, j = bonds[k].j;
        if (i < 0 || j < 0 || i >= b->n_sites || j >= b->n_sites || i == j)
            return fail(HPHI_ERR_INVALID_ARG, "bond %d (%d, %d) invalid for %d sites", k, i, j, b->n_sites);
        h->sbonds.push_back(bonds[k]);
        dev.push_back(Dev{i, j, bonds[k].jz, 0.5 * bonds[k].jxy});
    }
    if (dev.empty()) dev.push_back(Dev{0, 0, 0.0, 0.0});
    HPHI_TRY(upload(h->s_dbonds, dev.data(), sizeof(Dev) * dev.size()));
    if (hz) {
        h->s_hz.assign(hz, hz + b->n_sites);
        HPHI_TRY(upload(h->s_dhz, hz, sizeof(double) * b->n_sites));
    }
    if (d_ion) {
        h->s_dion.assign(d_ion, d_ion + b->n_sites);
        HPHI_TRY(upload(h->s_ddion, d_ion, sizeof(double) * b->n_sites));
    }
    HPHI_TRY(ham_ensure_reduce(h.get()));
    *out = h.release();
    return HPHI_OK;
}

} // extern "C"

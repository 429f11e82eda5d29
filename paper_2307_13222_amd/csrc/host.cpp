// Host-side pieces: error state, device memory, basis tables, tridiagonal
// eigensolver.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

#include "internal.h"

namespace hphi {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

const char *last_error() { return g_err.c_str(); }

int DevMem::alloc(size_t n)
{
    reset();
    if (n == 0) return HPHI_OK;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        return fail(HPHI_ERR_OUT_OF_MEMORY, "hipMalloc(%zu) failed: %s", n, hipGetErrorString(e));
    }
    bytes = n;
    return HPHI_OK;
}

void DevMem::reset()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

// Copies on the null stream and waits for them: a copy from pageable host
// memory may return before its data has landed, and kernels on the caller's
// streams (non-blocking ones do not order against the null stream) must
// see the data.
int upload(DevMem &m, const void *host, size_t bytes)
{
    HPHI_TRY(m.alloc(bytes));
    if (bytes) {
        HPHI_HIP(hipMemcpyAsync(m.p, host, bytes, hipMemcpyHostToDevice, nullptr));
        HPHI_HIP(hipStreamSynchronize(nullptr));
    }
    return HPHI_OK;
}

int zero_now(void *p, size_t bytes)
{
    HPHI_HIP(hipMemsetAsync(p, 0, bytes, nullptr));
    HPHI_HIP(hipStreamSynchronize(nullptr));
    return HPHI_OK;
}

static uint64_t binom_u64(int n, int k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    unsigned __int128 r = 1;
    for (int i = 1; i <= k; ++i) r = r * (unsigned)(n - k + i) / (unsigned)i;
    return (uint64_t)r;
}

// Two-level rank table. lo_rank[l] counts the n_lo-bit patterns below l with
// the same popcount; hi_off[h] counts sector states whose high part is below
// h, i.e. sum over h' < h of C(n_lo, n_pop - popcount(h')).
int build_species_tables(Species &s, int n_bits, int n_pop, int n_lo_override)
{
    if (n_bits < 1 || n_bits > 64 || n_pop < 0 || n_pop > n_bits)
        return fail(HPHI_ERR_INVALID_ARG, "invalid species (%d bits, %d set)", n_bits, n_pop);
    uint64_t dim = binom_u64(n_bits, n_pop);
    if (dim == 0) return fail(HPHI_ERR_EMPTY_SECTOR, "empty sector");
    if (dim > (uint64_t(1) << 62)) return fail(HPHI_ERR_DIM_OVERFLOW, "dimension beyond 2^62");
    int n_lo = n_lo_override > 0 ? n_lo_override : (n_bits + 1) / 2;
    if (n_lo > n_bits) n_lo = n_bits;
    int n_hi = n_bits - n_lo;
    if (n_lo > 24 || n_hi > 24)
        return fail(HPHI_ERR_DIM_OVERFLOW, "rank tables above 2^24 entries (%d bits)", n_bits);
    s.n_bits = n_bits; s.n_pop = n_pop; s.n_lo = n_lo; s.n_hi = n_hi; s.dim = (int64_t)dim;

    const uint32_t nl = 1u << n_lo, nh = 1u << n_hi;
    s.lo_rank.assign(nl, 0);
    s.lo_list.assign(nl, 0);
    s.lo_list_off.assign(n_lo + 2, 0);
    std::vector<uint32_t> cnt(n_lo + 1, 0);
    for (uint32_t l = 0; l < nl; ++l) s.lo_rank[l] = cnt[__builtin_popcount(l)]++;
    for (int k = 0; k <= n_lo; ++k) s.lo_list_off[k + 1] = s.lo_list_off[k] + cnt[k];
    for (uint32_t l = 0; l < nl; ++l)
        s.lo_list[s.lo_list_off[__builtin_popcount(l)] + s.lo_rank[l]] = l;
    s.hi_off.assign((size_t)nh + 1, 0);
    uint64_t acc = 0;
    for (uint32_t h = 0; h < nh; ++h) {
        s.hi_off[h] = acc;
        acc += binom_u64(n_lo, n_pop - __builtin_popcount(h));
    }
    s.hi_off[nh] = acc;
    if (acc != dim) return fail(HPHI_ERR_DIM_OVERFLOW, "rank table mismatch");
    s.state_bytes = n_bits <= 32 ? 4 : 8;
    return HPHI_OK;
}

int build_species(Species &s, int n_bits, int n_pop, int n_lo_override, bool materialize)
{
    HPHI_TRY(build_species_tables(s, n_bits, n_pop, n_lo_override));
    const uint64_t dim = (uint64_t)s.dim;
    const uint32_t nl = 1u << s.n_lo, nh = 1u << s.n_hi;
    HPHI_TRY(upload(s.d_lo_rank, s.lo_rank.data(), sizeof(uint32_t) * nl));
    HPHI_TRY(upload(s.d_hi_off, s.hi_off.data(), sizeof(uint64_t) * ((size_t)nh + 1)));
    if (dim < (uint64_t(1) << 32)) {
        std::vector<uint32_t> h32(s.hi_off.begin(), s.hi_off.end());
        HPHI_TRY(upload(s.d_hi_off32, h32.data(), sizeof(uint32_t) * h32.size()));
    }
    HPHI_TRY(upload(s.d_lo_list, s.lo_list.data(), sizeof(uint32_t) * nl));
    HPHI_TRY(upload(s.d_lo_list_off, s.lo_list_off.data(), sizeof(uint32_t) * s.lo_list_off.size()));
    if (materialize) {
        HPHI_TRY(s.d_states.alloc((size_t)dim * s.state_bytes));
        HPHI_TRY(launch_materialize(s, nullptr));
        HPHI_HIP(hipDeviceSynchronize());
    }
    return HPHI_OK;
}

uint64_t Species::state_at(int64_t r) const
{
    // last h with hi_off[h] <= r; it has a non-empty block because
    // hi_off[h + 1] > r there.
    auto it = std::upper_bound(hi_off.begin(), hi_off.end() - 1, (uint64_t)r);
    uint32_t h = (uint32_t)(it - hi_off.begin()) - 1;
    int k = n_pop - __builtin_popcount(h);
    uint32_t l = lo_list[lo_list_off[k] + (uint32_t)((uint64_t)r - hi_off[h])];
    return ((uint64_t)h << n_lo) | l;
}

int64_t Species::rank_of(uint64_t x) const
{
    if (n_bits < 64 && (x >> n_bits)) return -1;
    if (__builtin_popcountll(x) != n_pop) return -1;
    uint64_t lo = x & ((uint64_t(1) << n_lo) - 1);
    return (int64_t)(hi_off[x >> n_lo] + lo_rank[lo]);
}

int dtype_size(int dt)
{
    switch (dt) {
    case HPHI_F64: return 8;
    case HPHI_F32: return 4;
    case HPHI_C128: return 8;
    case HPHI_C64: return 4;
    }
    return 0;
}
int dtype_lanes(int dt) { return (dt == HPHI_C128 || dt == HPHI_C64) ? 2 : 1; }
bool dtype_is_f32(int dt) { return dt == HPHI_F32 || dt == HPHI_C64; }

// ------------------------------------------------------------ tridiagonal --
// Symmetric tridiagonal T: diagonal a[0..n), off-diagonal b[1..n) (b[i]
// couples i-1 and i). Eigenvalues by Sturm-sequence bisection (Barth,
// Martin, Wilkinson 1967): the number of negative pivots of the LDL^T
// factorization of T - x I equals the number of eigenvalues below x.

static int sturm_count(const double *a, const double *b2, int n, double x, double pivmin)
{
    int c = 0;
    double d = a[0] - x;
    if (std::fabs(d) < pivmin) d = -pivmin;
    if (d < 0) ++c;
    for (int i = 1; i < n; ++i) {
        d = a[i] - x - b2[i] / d;
        if (std::fabs(d) < pivmin) d = -pivmin;
        if (d < 0) ++c;
    }
    return c;
}

// Inverse iteration for the eigenvector of eigenvalue lam: solve
// (T - lam I) y = x by Gaussian elimination with partial pivoting on the
// tridiagonal band, three sweeps from a fixed start vector.
static void inverse_iteration(const double *a, const double *b, int n, double lam, double tnorm,
                              double *vec)
{
    std::vector<double> dl(n), d(n), du(n), du2(n), y(n);
    for (int i = 0; i < n; ++i) vec[i] = 1.0 / std::sqrt((double)n) * (1.0 + 0.01 * (i % 7));
    double shift = lam + 4.0 * std::numeric_limits<double>::epsilon() * tnorm;
    for (int sweep = 0; sweep < 3; ++sweep) {
        for (int i = 0; i < n; ++i) {
            d[i] = a[i] - shift;
            du[i] = (i + 1 < n) ? b[i + 1] : 0.0;
            dl[i] = (i + 1 < n) ? b[i + 1] : 0.0;
            du2[i] = 0.0;
            y[i] = vec[i];
        }
        // forward elimination with row interchanges (LAPACK dgtsv scheme)
        for (int i = 0; i + 1 < n; ++i) {
            if (std::fabs(d[i]) >= std::fabs(dl[i])) {
                double piv = d[i];
                if (piv == 0.0) piv = d[i] = 1e-300;
                double f = dl[i] / piv;
                d[i + 1] -= f * du[i];
                y[i + 1] -= f * y[i];
                du2[i] = 0.0;
            } else {
                double f = d[i] / dl[i];
                d[i] = dl[i];
                double t = d[i + 1];
                d[i + 1] = du[i] - f * t;
                if (i + 2 < n) {
                    du2[i] = du[i + 1];
                    du[i + 1] = -f * du2[i];
                }
                du[i] = t;
                double ty = y[i];
                y[i] = y[i + 1];
                y[i + 1] = ty - f * y[i + 1];
            }
        }
        if (d[n - 1] == 0.0) d[n - 1] = 1e-300;
        // back substitution
        y[n - 1] /= d[n - 1];
        if (n > 1) y[n - 2] = (y[n - 2] - du[n - 2] * y[n - 1]) / d[n - 2];
        for (int i = n - 3; i >= 0; --i) y[i] = (y[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / d[i];
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += y[i] * y[i];
        nrm = std::sqrt(nrm);
        for (int i = 0; i < n; ++i) vec[i] = y[i] / nrm;
    }
    // fixed sign: largest-magnitude component positive
    int im = 0;
    for (int i = 1; i < n; ++i)
        if (std::fabs(vec[i]) > std::fabs(vec[im])) im = i;
    if (vec[im] < 0)
        for (int i = 0; i < n; ++i) vec[i] = -vec[i];
}

int tridiag_lowest(const double *a, const double *b, int n, int k, double *eig, double *vec)
{
    if (n < 1 || k < 1 || k > n || !a || !b || !eig)
        return fail(HPHI_ERR_INVALID_ARG, "tridiag: n=%d k=%d", n, k);
    std::vector<double> b2(n, 0.0);
    double lo = a[0], hi = a[0], tnorm = 0.0;
    for (int i = 0; i < n; ++i) {
        double r = (i > 0 ? std::fabs(b[i]) : 0.0) + (i + 1 < n ? std::fabs(b[i + 1]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
        if (i > 0) b2[i] = b[i] * b[i];
        tnorm = std::max(tnorm, std::fabs(a[i]) + r);
    }
    const double eps = std::numeric_limits<double>::epsilon();
    double pivmin = std::max(std::numeric_limits<double>::min(), eps * eps * tnorm * tnorm * 1e-3);
    lo -= 2 * eps * tnorm + pivmin;
    hi += 2 * eps * tnorm + pivmin;
    for (int j = 0; j < k; ++j) {
        double l = lo, h = hi;
        for (int it = 0; it < 200; ++it) {
            double m = 0.5 * (l + h);
            if (m <= l || m >= h) break;
            if (h - l <= 2 * eps * std::max(std::fabs(l), std::fabs(h)) + pivmin) break;
            if (sturm_count(a, b2.data(), n, m, pivmin) > j) h = m; else l = m;
        }
        eig[j] = 0.5 * (l + h);
    }
    if (vec) inverse_iteration(a, b, n, eig[0], tnorm, vec);
    return HPHI_OK;
}

} // namespace hphi

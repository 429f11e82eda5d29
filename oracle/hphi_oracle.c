/*
 * Oracle for the H*v hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct CPU code. Only tests/, the smoke check and
 * the CPU-baseline leg of the benchmark may load it. It shares nothing with
 * the HIP library (no headers, no tables, no helpers).
 *
 * What it computes (HPhi update paper, arXiv:2307.13222):
 *   - the sector basis: every N-bit configuration with a fixed number of set
 *     bits (fixed total S^z for spins, fixed N_up / N_dn for electrons), the
 *     sector keywords 2Sz / nelec of the Standard-mode tables (Sec. 4.1,
 *     Table "Keywords"; the cTPQ basics of Sec. 3.5.1 describe x as the set of
 *     spin or particle positions);
 *   - the spin-1/2 XXZ Hamiltonian applied to a vector, row by row
 *     (Heisenberg model of Sec. 3.2, S^z = (n_up - n_dn)/2);
 *   - the spin-1/2 XYZ Hamiltonian with transverse and longitudinal fields
 *     on the full 2^N space (SpinGC of Sec. 4.1), Pauli by Pauli;
 *   - the spin-S Heisenberg Hamiltonian with total S^z conserved (keyword
 *     2S of Sec. 4.1) from the ladder-operator matrix elements;
 *   - the Hubbard Hamiltonian -t sum c^+c + U n_up n_dn applied to a vector
 *     (Sec. 3.4, Eq. Hquench; Sec. 5 transfer integrals), with the fermion
 *     sign written out from the anticommutation relations, and the two-body
 *     terms of Sec. 5, Eq. ham_general (inter-site Coulomb, Hund, exchange,
 *     pair hopping), applied operator by operator;
 *
 * Readings where the paper is silent (bit 1 = up spin / occupied orbital,
 * ascending integer order, all up orbitals ordered before all down orbitals)
 * are fixed here in the simplest form and are stated again where used.
 *
 * Ranking is done two independent ways: binary search in the sorted list,
 * and the combinatorial number system (rank = sum_k C(c_k, k) over the set
 * bit positions c_1 < ... < c_n), which equals the ascending position.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

static int pc64(uint64_t x) { return __builtin_popcountll(x); }

/* Binomial coefficient C(n, k) by the multiplicative formula (exact while it
 * fits in 64 bits; every use here is far below that). */
uint64_t or_binom(int n, int k)
{
    if (k < 0 || n < 0 || k > n) return 0;
    if (k > n - k) k = n - k;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

/* All nbits-bit integers with popcount npop, ascending. Brute force over
 * [0, 2^nbits). Returns the count written (at most cap). */
int64_t or_basis_fill(int nbits, int npop, uint64_t *out, int64_t cap)
{
    int64_t n = 0;
    uint64_t end = (nbits >= 64) ? 0 : ((uint64_t)1 << nbits);
    for (uint64_t x = 0; x < end; ++x) {
        if (pc64(x) == npop) {
            if (n < cap) out[n] = x;
            ++n;
        }
    }
    return n;
}

/* Combinatorial-number-system rank: sum over the set bits, taken from the
 * lowest (k = 1) to the highest (k = n), of C(position, k). */
int64_t or_rank_combinadic(uint64_t x)
{
    int64_t r = 0;
    int k = 0;
    for (int pos = 0; pos < 64; ++pos) {
        if ((x >> pos) & 1) {
            ++k;
            r += (int64_t)or_binom(pos, k);
        }
    }
    return r;
}

/* Inverse of the above: the configuration with npop set bits whose rank is r.
 * Greedy from the highest set bit down. */
uint64_t or_unrank_combinadic(int64_t r, int npop)
{
    uint64_t x = 0;
    for (int k = npop; k >= 1; --k) {
        int pos = k - 1;
        while ((int64_t)or_binom(pos + 1, k) <= r) ++pos;
        r -= (int64_t)or_binom(pos, k);
        x |= (uint64_t)1 << pos;
    }
    return x;
}

/* Position of x in the ascending list, or -1. */
int64_t or_rank_search(const uint64_t *list, int64_t dim, uint64_t x)
{
    int64_t lo = 0, hi = dim - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (list[mid] == x) return mid;
        if (list[mid] < x) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

void or_rank_search_many(const uint64_t *list, int64_t dim, const uint64_t *xs,
                         int64_t n, int64_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = or_rank_search(list, dim, xs[i]);
}

void or_rank_combinadic_many(const uint64_t *xs, int64_t n, int64_t *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = or_rank_combinadic(xs[i]);
}

/* ---------------------------------------------------------------- spins -- */

/* One matrix row of the spin-1/2 XXZ Hamiltonian
 *   H = sum_b [ Jz_b S^z_i S^z_j + Jxy_b (S^x_i S^x_j + S^y_i S^y_j) ]
 *       - sum_i h_i S^z_i,
 * bit 1 = up spin (S^z = +1/2). S^x S^x + S^y S^y = (S^+S^- + S^-S^+)/2, so a
 * bond whose two spins are antiparallel connects x to x with both spins
 * flipped, with amplitude Jxy/2. The diagonal is Jz/4 for a parallel pair
 * and -Jz/4 for an antiparallel one. Emits (column configuration, value)
 * pairs: the diagonal first, then one entry per antiparallel bond. */
static int spin_row(uint64_t x, int nsites, int nb, const int32_t *bi,
                    const int32_t *bj, const double *jz, const double *jxy,
                    const double *hz, uint64_t *cols, double *vals)
{
    double d = 0.0;
    int m = 1;
    for (int b = 0; b < nb; ++b) {
        int si = (int)((x >> bi[b]) & 1), sj = (int)((x >> bj[b]) & 1);
        if (si == sj) {
            d += 0.25 * jz[b];
        } else {
            d -= 0.25 * jz[b];
            cols[m] = x ^ (((uint64_t)1 << bi[b]) | ((uint64_t)1 << bj[b]));
            vals[m] = 0.5 * jxy[b];
            ++m;
        }
    }
    if (hz) {
        for (int i = 0; i < nsites; ++i) {
            double sz = ((x >> i) & 1) ? 0.5 : -0.5;
            d -= hz[i] * sz;
        }
    }
    cols[0] = x;
    vals[0] = d;
    return m;
}

/* w = H v over a materialized ascending basis; ranks by binary search. */
void or_spin_hv(int nsites, const uint64_t *states, int64_t dim, int nb,
                const int32_t *bi, const int32_t *bj, const double *jz,
                const double *jxy, const double *hz, const double *v,
                double *w)
{
    #pragma omp parallel
    {
        uint64_t *cols = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
        double *vals = (double *)malloc(sizeof(double) * (size_t)(nb + 1));
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < dim; ++r) {
            int m = spin_row(states[r], nsites, nb, bi, bj, jz, jxy, hz, cols, vals);
            double acc = vals[0] * v[r];
            for (int k = 1; k < m; ++k) {
                int64_t c = or_rank_search(states, dim, cols[k]);
                acc += vals[k] * v[c];
            }
            w[r] = acc;
        }
        free(cols);
        free(vals);
    }
}

/* One sparse row by index, without a materialized basis (combinadic rank).
 * For sampled-row checks at sizes whose basis list does not fit in memory.
 * Returns the number of entries (diagonal first). */
int or_spin_row_by_index(int nsites, int npop, int64_t row, int nb,
                         const int32_t *bi, const int32_t *bj, const double *jz,
                         const double *jxy, const double *hz, int64_t *cols,
                         double *vals)
{
    uint64_t x = or_unrank_combinadic(row, npop);
    uint64_t *cfg = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
    int m = spin_row(x, nsites, nb, bi, bj, jz, jxy, hz, cfg, vals);
    for (int k = 0; k < m; ++k) cols[k] = or_rank_combinadic(cfg[k]);
    free(cfg);
    return m;
}

/* Diagonal S^z_l for each site of each configuration, used by the S^z(q)
 * excitation: sz[r * nsites + l] = +1/2 or -1/2. */
void or_spin_sz_table(int nsites, const uint64_t *states, int64_t dim, double *sz)
{
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < dim; ++r)
        for (int l = 0; l < nsites; ++l)
            sz[r * nsites + l] = ((states[r] >> l) & 1) ? 0.5 : -0.5;
}

/* -------------------------------------------------------------- Hubbard -- */

/* Fermion sign of c^+_a c_b (a != b, same species) acting on a configuration
 * occ in which b is occupied and a is empty, for the ordering
 * |occ> = prod_{k in occ, ascending} c^+_k |0>.
 * c_b anticommutes past the occupied orbitals below b; c^+_a then moves to
 * its sorted place past the occupied orbitals (b removed) below a. The sign
 * is (-1)^(number of those crossings), computed here literally. */
static double hop_sign(uint64_t occ, int a, int b)
{
    int below_b = 0, below_a = 0;
    for (int k = 0; k < b; ++k) below_b += (int)((occ >> k) & 1);
    uint64_t rest = occ & ~((uint64_t)1 << b);
    for (int k = 0; k < a; ++k) below_a += (int)((rest >> k) & 1);
    return ((below_a + below_b) & 1) ? -1.0 : 1.0;
}

/* w = H v for
 *   H = - sum_h t_h sum_sigma (c^+_{i sigma} c_{j sigma} + c^+_{j sigma} c_{i sigma})
 *       + sum_i U_i n_{i up} n_{i dn}.
 * Basis index = r_up * dim_dn + r_dn (up-major). All up orbitals precede all
 * down orbitals in the operator ordering; a same-species hop then moves past
 * the other species an even number of times in total, so only the
 * same-species crossings give a sign. */
void or_hubbard_hv(int nsites, const uint64_t *ups, int64_t dup,
                   const uint64_t *dns, int64_t ddn, int nh, const int32_t *hi,
                   const int32_t *hj, const double *ht, const double *u_site,
                   const double *v, double *w)
{
    (void)nsites;
    #pragma omp parallel for schedule(static)
    for (int64_t ru = 0; ru < dup; ++ru) {
        uint64_t u = ups[ru];
        for (int64_t rd = 0; rd < ddn; ++rd) {
            uint64_t d = dns[rd];
            int64_t me = ru * ddn + rd;
            double diag = 0.0;
            for (int i = 0; i < nsites; ++i)
                if (((u >> i) & 1) && ((d >> i) & 1)) diag += u_site[i];
            double acc = diag * v[me];
            for (int h = 0; h < nh; ++h) {
                int i = hi[h], j = hj[h];
                /* up species */
                int ui = (int)((u >> i) & 1), uj = (int)((u >> j) & 1);
                if (ui != uj) {
                    int a = ui ? j : i, b = ui ? i : j;   /* move b -> a */
                    uint64_t u2 = u ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
                    int64_t c = or_rank_search(ups, dup, u2);
                    /* <u2| c^+_a c_b |u> = sign; element of H is -t * sign */
                    acc += -ht[h] * hop_sign(u, a, b) * v[c * ddn + rd];
                }
                int di = (int)((d >> i) & 1), dj = (int)((d >> j) & 1);
                if (di != dj) {
                    int a = di ? j : i, b = di ? i : j;
                    uint64_t d2 = d ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
                    int64_t c = or_rank_search(dns, ddn, d2);
                    acc += -ht[h] * hop_sign(d, a, b) * v[ru * ddn + c];
                }
            }
            w[me] = acc;
        }
    }
}

/* Rows [ru_first, ru_first + ru_count) x all r_dn of w = H v (the same
 * arithmetic as or_hubbard_hv, on a bounded set of output rows; v is the
 * whole vector). w holds ru_count * ddn entries. */
void or_hubbard_hv_rows(int nsites, const uint64_t *ups, int64_t dup,
                        const uint64_t *dns, int64_t ddn, int nh, const int32_t *hi,
                        const int32_t *hj, const double *ht, const double *u_site,
                        const double *v, int64_t ru_first, int64_t ru_count, double *w)
{
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < ru_count * ddn; ++k) {
        int64_t ru = ru_first + k / ddn, rd = k % ddn;
        uint64_t u = ups[ru], d = dns[rd];
        double diag = 0.0;
        for (int i = 0; i < nsites; ++i)
            if (((u >> i) & 1) && ((d >> i) & 1)) diag += u_site[i];
        double acc = diag * v[ru * ddn + rd];
        for (int h = 0; h < nh; ++h) {
            int i = hi[h], j = hj[h];
            int ui = (int)((u >> i) & 1), uj = (int)((u >> j) & 1);
            if (ui != uj) {
                int a = ui ? j : i, b = ui ? i : j;
                uint64_t u2 = u ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
                acc += -ht[h] * hop_sign(u, a, b) * v[or_rank_search(ups, dup, u2) * ddn + rd];
            }
            int di = (int)((d >> i) & 1), dj = (int)((d >> j) & 1);
            if (di != dj) {
                int a = di ? j : i, b = di ? i : j;
                uint64_t d2 = d ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
                acc += -ht[h] * hop_sign(d, a, b) * v[ru * ddn + or_rank_search(dns, ddn, d2)];
            }
        }
        w[k] = acc;
    }
}

/* One sparse row of the Hubbard Hamiltonian by (r_up, r_dn); entries are
 * flat indices. Returns the count (diagonal first). */
int or_hubbard_row(int nsites, const uint64_t *ups, int64_t dup,
                   const uint64_t *dns, int64_t ddn, int nh, const int32_t *hi,
                   const int32_t *hj, const double *ht, const double *u_site,
                   int64_t ru, int64_t rd, int64_t *cols, double *vals)
{
    (void)nsites;
    uint64_t u = ups[ru], d = dns[rd];
    double diag = 0.0;
    for (int i = 0; i < nsites; ++i)
        if (((u >> i) & 1) && ((d >> i) & 1)) diag += u_site[i];
    int m = 0;
    cols[m] = ru * ddn + rd; vals[m] = diag; ++m;
    for (int h = 0; h < nh; ++h) {
        int i = hi[h], j = hj[h];
        int ui = (int)((u >> i) & 1), uj = (int)((u >> j) & 1);
        if (ui != uj) {
            int a = ui ? j : i, b = ui ? i : j;
            uint64_t u2 = u ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
            cols[m] = or_rank_search(ups, dup, u2) * ddn + rd;
            vals[m] = -ht[h] * hop_sign(u, a, b);
            ++m;
        }
        int di = (int)((d >> i) & 1), dj = (int)((d >> j) & 1);
        if (di != dj) {
            int a = di ? j : i, b = di ? i : j;
            uint64_t d2 = d ^ (((uint64_t)1 << i) | ((uint64_t)1 << j));
            cols[m] = ru * ddn + or_rank_search(dns, ddn, d2);
            vals[m] = -ht[h] * hop_sign(d, a, b);
            ++m;
        }
    }
    return m;
}

/* ----------------------------------------------------------- spin-S -- */

/* Spin-S sites (2S+1 levels; keyword 2S of Sec. 4.1, "Remarks on the keyword
 * model"): site i holds m_i = S^z_i + S in {0, ..., 2S}, stored in bits
 * [i b, (i + 1) b) of the configuration, b the fewest bits that hold 2S. */
static int spin_s_bits(int two_s) { int b = 1; while ((1 << b) <= two_s) ++b; return b; }

static int cmp_u64(const void *a, const void *b)
{
    const uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* All configurations with digits <= 2S and digit sum msum, ascending.
 * Brute force over the (2S+1)^N digit strings. Returns the count (at most
 * cap written). */
int64_t or_spin_s_basis_fill(int nsites, int two_s, int msum, uint64_t *out, int64_t cap)
{
    const int b = spin_s_bits(two_s);
    int digits[64];
    for (int i = 0; i < nsites; ++i) digits[i] = 0;
    int64_t n = 0;
    /* odometer over digit strings, site 0 fastest */
    for (;;) {
        int sum = 0;
        for (int i = 0; i < nsites; ++i) sum += digits[i];
        if (sum == msum) {
            uint64_t x = 0;
            for (int i = 0; i < nsites; ++i) x |= (uint64_t)digits[i] << (i * b);
            if (n < cap) out[n] = x;
            ++n;
        }
        int i = 0;
        while (i < nsites && digits[i] == two_s) digits[i++] = 0;
        if (i == nsites) break;
        ++digits[i];
    }
    /* the odometer visits digit strings in an order that is not the
     * numeric one; sort what was written */
    int64_t m = n < cap ? n : cap;
    qsort(out, (size_t)m, sizeof(uint64_t), cmp_u64);
    return n;
}

/* <s +- 1| S^+- |s> for spin S (s = m - S): sqrt(S(S+1) - s(s +- 1)). */
static double ladder_amp(int two_s, int m, int up)
{
    const double S = 0.5 * two_s, sz = m - S;
    return sqrt(S * (S + 1.0) - sz * (sz + (up ? 1.0 : -1.0)));
}

/* One row of the spin-S Hamiltonian with total S^z conserved:
 *   H = sum_b [jz S^z_i S^z_j + jxy/2 (S^+_i S^-_j + S^-_i S^+_j)]
 *       - sum_i hz_i S^z_i + sum_i d_i (S^z_i)^2.
 * Columns by binary search in the sorted state list. Returns the count. */
int or_spin_s_row(int nsites, int two_s, const uint64_t *states, int64_t dim, int nb, const int32_t *bi,
                  const int32_t *bj, const double *jz, const double *jxy, const double *hz, const double *dion,
                  int64_t r, int64_t *cols, double *vals)
{
    const int b = spin_s_bits(two_s);
    const uint64_t dmask = ((uint64_t)1 << b) - 1;
    const uint64_t x = states[r];
    const double S = 0.5 * two_s;
    double diag = 0.0;
    int m = 1;
    for (int k = 0; k < nb; ++k) {
        const int i = bi[k], j = bj[k];
        const int mi = (int)((x >> (i * b)) & dmask), mj = (int)((x >> (j * b)) & dmask);
        diag += jz[k] * (mi - S) * (mj - S);
        if (jxy[k] == 0.0) continue;
        /* S^+_i S^-_j */
        if (mi < two_s && mj > 0) {
            uint64_t y = x + ((uint64_t)1 << (i * b)) - ((uint64_t)1 << (j * b));
            cols[m] = or_rank_search(states, dim, y);
            vals[m] = 0.5 * jxy[k] * ladder_amp(two_s, mi, 1) * ladder_amp(two_s, mj, 0);
            ++m;
        }
        /* S^-_i S^+_j */
        if (mi > 0 && mj < two_s) {
            uint64_t y = x - ((uint64_t)1 << (i * b)) + ((uint64_t)1 << (j * b));
            cols[m] = or_rank_search(states, dim, y);
            vals[m] = 0.5 * jxy[k] * ladder_amp(two_s, mi, 0) * ladder_amp(two_s, mj, 1);
            ++m;
        }
    }
    for (int i = 0; i < nsites; ++i) {
        const double sz = (double)((x >> (i * b)) & dmask) - S;
        if (hz) diag -= hz[i] * sz;
        if (dion) diag += dion[i] * sz * sz;
    }
    cols[0] = r;
    vals[0] = diag;
    return m;
}

void or_spin_s_hv(int nsites, int two_s, const uint64_t *states, int64_t dim, int nb, const int32_t *bi,
                  const int32_t *bj, const double *jz, const double *jxy, const double *hz, const double *dion,
                  const double *v, double *w)
{
    #pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(1 + 2 * nb));
        double *vals = (double *)malloc(sizeof(double) * (size_t)(1 + 2 * nb));
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < dim; ++r) {
            int m = or_spin_s_row(nsites, two_s, states, dim, nb, bi, bj, jz, jxy, hz, dion, r, cols, vals);
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += vals[k] * v[cols[k]];
            w[r] = acc;
        }
        free(cols);
        free(vals);
    }
}

void or_spin_s_ell(int nsites, int two_s, const uint64_t *states, int64_t dim, int nb, const int32_t *bi,
                   const int32_t *bj, const double *jz, const double *jxy, const double *hz, const double *dion,
                   int64_t *cols, double *vals, int32_t *count)
{
    const int64_t stride = 1 + 2 * (int64_t)nb;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < dim; ++r)
        count[r] = or_spin_s_row(nsites, two_s, states, dim, nb, bi, bj, jz, jxy, hz, dion, r, cols + r * stride,
                                 vals + r * stride);
}

/* ----------------------------------------------------------- SpinGC -- */

/* Pauli matrix sigma^a (a = 0: x, 1: y, 2: z) on site i applied to the
 * configuration x (bit 1 = up): returns x' and the amplitude
 * <x'| sigma^a_i |x> = re + i im. In the basis (up, down),
 * sigma^x = [[0, 1], [1, 0]], sigma^y = [[0, -i], [i, 0]],
 * sigma^z = [[1, 0], [0, -1]]. */
static uint64_t pauli_apply(int a, int i, uint64_t x, double *re, double *im)
{
    const int up = (int)((x >> i) & 1);
    if (a == 2) {
        *re = up ? 1.0 : -1.0;
        *im = 0.0;
        return x;
    }
    const uint64_t y = x ^ ((uint64_t)1 << i);
    if (a == 0) {
        *re = 1.0;
        *im = 0.0;
    } else {
        /* column up -> (0, i): the down component gets +i; column down ->
         * (-i, 0): the up component gets -i */
        *re = 0.0;
        *im = up ? 1.0 : -1.0;
    }
    return y;
}

/* One row of the spin-1/2 Hamiltonian on the full 2^N space (SpinGC model
 * keyword, Sec. 4.1 Table "Keywords": no S^z conservation):
 *   H = sum_b [jx S^x_i S^x_j + jy S^y_i S^y_j + jz S^z_i S^z_j]
 *       - sum_i (hx_i S^x_i + hz_i S^z_i),   S^a = sigma^a / 2.
 * Every product is applied Pauli by Pauli; the index of a configuration is
 * the configuration itself. Entries: diagonal first, then one per
 * off-diagonal term (a target may repeat). Returns the count. */
int or_spin_gc_row(int nsites, int nb, const int32_t *bi, const int32_t *bj, const double *jx,
                   const double *jy, const double *jz, const double *hx, const double *hz,
                   uint64_t x, int64_t *cols, double *vals)
{
    double diag = 0.0;
    int m = 1;
    for (int b = 0; b < nb; ++b) {
        const double jab[3] = {jx[b], jy[b], jz[b]};
        for (int a = 0; a < 3; ++a) {
            if (jab[a] == 0.0) continue;
            double r1, i1, r2, i2;
            uint64_t y = pauli_apply(a, bj[b], x, &r1, &i1);
            y = pauli_apply(a, bi[b], y, &r2, &i2);
            const double re = r1 * r2 - i1 * i2;   /* the imaginary part cancels */
            const double val = 0.25 * jab[a] * re;
            if (y == x) diag += val;
            else { cols[m] = (int64_t)y; vals[m] = val; ++m; }
        }
    }
    for (int i = 0; i < nsites; ++i) {
        double re, im;
        if (hx && hx[i] != 0.0) {
            uint64_t y = pauli_apply(0, i, x, &re, &im);
            cols[m] = (int64_t)y; vals[m] = -0.5 * hx[i] * re; ++m;
        }
        if (hz && hz[i] != 0.0) {
            pauli_apply(2, i, x, &re, &im);
            diag += -0.5 * hz[i] * re;
        }
    }
    cols[0] = (int64_t)x;
    vals[0] = diag;
    return m;
}

/* w = H v on the full space (every row through or_spin_gc_row). */
void or_spin_gc_hv(int nsites, int nb, const int32_t *bi, const int32_t *bj, const double *jx,
                   const double *jy, const double *jz, const double *hx, const double *hz,
                   const double *v, double *w)
{
    const int64_t dim = (int64_t)1 << nsites;
    const int cap = 1 + 3 * nb + nsites;
    #pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *vals = (double *)malloc(sizeof(double) * (size_t)cap);
        #pragma omp for schedule(static)
        for (int64_t x = 0; x < dim; ++x) {
            int m = or_spin_gc_row(nsites, nb, bi, bj, jx, jy, jz, hx, hz, (uint64_t)x, cols, vals);
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += vals[k] * v[cols[k]];
            w[x] = acc;
        }
        free(cols);
        free(vals);
    }
}

/* Rows [first, first + count) of H v; w holds count entries. */
void or_spin_gc_hv_rows(int nsites, int nb, const int32_t *bi, const int32_t *bj, const double *jx,
                        const double *jy, const double *jz, const double *hx, const double *hz,
                        const double *v, int64_t first, int64_t count, double *w)
{
    const int cap = 1 + 3 * nb + nsites;
    #pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
        double *vals = (double *)malloc(sizeof(double) * (size_t)cap);
        #pragma omp for schedule(static)
        for (int64_t k = 0; k < count; ++k) {
            int m = or_spin_gc_row(nsites, nb, bi, bj, jx, jy, jz, hx, hz, (uint64_t)(first + k), cols, vals);
            double acc = 0.0;
            for (int q = 0; q < m; ++q) acc += vals[q] * v[cols[q]];
            w[k] = acc;
        }
        free(cols);
        free(vals);
    }
}

/* Every row in a fixed-stride layout (stride 1 + 3 nb + nsites). */
void or_spin_gc_ell(int nsites, int nb, const int32_t *bi, const int32_t *bj, const double *jx,
                    const double *jy, const double *jz, const double *hx, const double *hz,
                    int64_t *cols, double *vals, int32_t *count)
{
    const int64_t dim = (int64_t)1 << nsites;
    const int64_t stride = 1 + 3 * (int64_t)nb + nsites;
    #pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < dim; ++x)
        count[x] = or_spin_gc_row(nsites, nb, bi, bj, jx, jy, jz, hx, hz, (uint64_t)x, cols + x * stride,
                                  vals + x * stride);
}

/* ------------------------------------------------ Hubbard two-body terms -- */

/* One creation (dag = 1) or annihilation (dag = 0) operator on orbital o of
 * the occupation pattern occ over 2 * nsites orbitals (orbital i = site i
 * up, nsites + i = site i down), with |occ> = prod_{o in occ, ascending}
 * c^+_o |0>. The operator anticommutes past every occupied orbital below o
 * before it acts, so the amplitude picks up (-1)^(that count). Returns 0
 * when the result vanishes (c^+ on an occupied or c on an empty orbital). */
static int apply_fermion(uint64_t *occ, int o, int dag, double *sign)
{
    int occupied = (int)((*occ >> o) & 1);
    if (dag == occupied) return 0;
    int below = 0;
    for (int k = 0; k < o; ++k) below += (int)((*occ >> k) & 1);
    if (below & 1) *sign = -*sign;
    *occ ^= (uint64_t)1 << o;
    return 1;
}

/* An operator product c^(d0)_{o0} c^(d1)_{o1} c^(d2)_{o2} c^(d3)_{o3} applied
 * to occ, rightmost factor first. */
static int apply_string4(uint64_t *occ, const int *orb, const int *dag, double *sign)
{
    for (int k = 3; k >= 0; --k)
        if (!apply_fermion(occ, orb[k], dag[k], sign)) return 0;
    return 1;
}

/* Two-body part of one row (Sec. 5, Eq. ham_general, one coefficient set per
 * listed site pair p = (i, j), i != j):
 *   V_p n_i n_j - JH_p (n_i,up n_j,up + n_i,dn n_j,dn)        (n_i = n_i,up + n_i,dn)
 *   + JX_p (c+_i,up c_j,up c+_j,dn c_i,dn + h.c.)           (exchange)
 *   + JP_p (c+_i,up c_j,up c+_i,dn c_j,dn + h.c.)           (pair hopping)
 * The off-diagonal products and their conjugates are applied factor by
 * factor to the full occupation pattern, so every fermion sign comes from
 * the anticommutation relations alone. Entries are flat indices; the
 * diagonal comes first. Returns the count (at most 1 + 4 * np). */
int or_hubbard_pairs_row(int nsites, const uint64_t *ups, int64_t dup,
                         const uint64_t *dns, int64_t ddn, int np, const int32_t *pi,
                         const int32_t *pj, const double *pv, const double *pjh,
                         const double *pjx, const double *pjp, int64_t ru, int64_t rd,
                         int64_t *cols, double *vals)
{
    const uint64_t u = ups[ru], d = dns[rd];
    const uint64_t occ0 = u | (d << nsites);
    const uint64_t lowmask = (nsites >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << nsites) - 1);
    double diag = 0.0;
    for (int p = 0; p < np; ++p) {
        int i = pi[p], j = pj[p];
        int niu = (int)((u >> i) & 1), nid = (int)((d >> i) & 1);
        int nju = (int)((u >> j) & 1), njd = (int)((d >> j) & 1);
        diag += pv[p] * (double)((niu + nid) * (nju + njd));
        diag -= pjh[p] * (double)(niu * nju + nid * njd);
    }
    int m = 0;
    cols[m] = ru * ddn + rd; vals[m] = diag; ++m;
    for (int p = 0; p < np; ++p) {
        const int iu = pi[p], ju = pj[p], id = nsites + pi[p], jd = nsites + pj[p];
        /* exchange, its conjugate, pair hopping, its conjugate */
        const int orb[4][4] = {{iu, ju, jd, id}, {id, jd, ju, iu}, {iu, ju, id, jd}, {jd, id, ju, iu}};
        const int dag[4][4] = {{1, 0, 1, 0}, {1, 0, 1, 0}, {1, 0, 1, 0}, {1, 0, 1, 0}};
        const double coef[4] = {pjx[p], pjx[p], pjp[p], pjp[p]};
        for (int s = 0; s < 4; ++s) {
            if (coef[s] == 0.0) continue;
            uint64_t occ = occ0;
            double sign = 1.0;
            if (!apply_string4(&occ, orb[s], dag[s], &sign)) continue;
            uint64_t u2 = occ & lowmask, d2 = occ >> nsites;
            cols[m] = or_rank_search(ups, dup, u2) * ddn + or_rank_search(dns, ddn, d2);
            vals[m] = coef[s] * sign;
            ++m;
        }
    }
    return m;
}

/* w = H_2body v (every row through or_hubbard_pairs_row). */
void or_hubbard_pairs_hv(int nsites, const uint64_t *ups, int64_t dup,
                         const uint64_t *dns, int64_t ddn, int np, const int32_t *pi,
                         const int32_t *pj, const double *pv, const double *pjh,
                         const double *pjx, const double *pjp, const double *v, double *w)
{
    #pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(1 + 4 * np));
        double *vals = (double *)malloc(sizeof(double) * (size_t)(1 + 4 * np));
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < dup * ddn; ++r) {
            int m = or_hubbard_pairs_row(nsites, ups, dup, dns, ddn, np, pi, pj, pv, pjh, pjx, pjp,
                                         r / ddn, r % ddn, cols, vals);
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += vals[k] * v[cols[k]];
            w[r] = acc;
        }
        free(cols);
        free(vals);
    }
}

/* Rows [ru_first, ru_first + ru_count) x all r_dn of H_2body v (v is the
 * whole vector); w holds ru_count * ddn entries. */
void or_hubbard_pairs_hv_rows(int nsites, const uint64_t *ups, int64_t dup,
                              const uint64_t *dns, int64_t ddn, int np, const int32_t *pi,
                              const int32_t *pj, const double *pv, const double *pjh,
                              const double *pjx, const double *pjp, const double *v,
                              int64_t ru_first, int64_t ru_count, double *w)
{
    #pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(1 + 4 * np));
        double *vals = (double *)malloc(sizeof(double) * (size_t)(1 + 4 * np));
        #pragma omp for schedule(static)
        for (int64_t k = 0; k < ru_count * ddn; ++k) {
            int m = or_hubbard_pairs_row(nsites, ups, dup, dns, ddn, np, pi, pj, pv, pjh, pjx, pjp,
                                         ru_first + k / ddn, k % ddn, cols, vals);
            double acc = 0.0;
            for (int q = 0; q < m; ++q) acc += vals[q] * v[cols[q]];
            w[k] = acc;
        }
        free(cols);
        free(vals);
    }
}

/* Every row of H_2body in a fixed-stride layout (stride 1 + 4 * np). */
void or_hubbard_pairs_ell(int nsites, const uint64_t *ups, int64_t dup,
                          const uint64_t *dns, int64_t ddn, int np, const int32_t *pi,
                          const int32_t *pj, const double *pv, const double *pjh,
                          const double *pjx, const double *pjp, int64_t *cols, double *vals,
                          int32_t *count)
{
    int64_t stride = 1 + 4 * (int64_t)np;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < dup * ddn; ++r)
        count[r] = or_hubbard_pairs_row(nsites, ups, dup, dns, ddn, np, pi, pj, pv, pjh, pjx, pjp,
                                        r / ddn, r % ddn, cols + r * stride, vals + r * stride);
}

/* --------------------------------------------------------------- random -- */

/* SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state
 * passed through the published finalizer. Element i of the stream for a seed
 * is the output after i+1 advances, so any element can be made directly. */
static uint64_t splitmix_out(uint64_t state)
{
    uint64_t z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void or_splitmix_u64(uint64_t seed, int64_t first, int64_t n, uint64_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = splitmix_out(seed + (uint64_t)(first + i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Uniform on [-1/2, 1/2): the top 53 bits scaled by 2^-53, minus 1/2. */
void or_splitmix_uniform(uint64_t seed, int64_t first, int64_t n, double *out)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        uint64_t z = splitmix_out(seed + (uint64_t)(first + i + 1) * 0x9E3779B97F4A7C15ULL);
        out[i] = (double)(z >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
}

/* ------------------------------------------------------ sparse export -- */

/* Every row of the spin Hamiltonian in a fixed-stride layout (stride nb+1):
 * cols[r*(nb+1)+k], vals[...], count[r]. Used to form a sparse matrix for
 * direct solves and dense checks at small sizes. */
void or_spin_ell(int nsites, const uint64_t *states, int64_t dim, int nb,
                 const int32_t *bi, const int32_t *bj, const double *jz,
                 const double *jxy, const double *hz, int64_t *cols,
                 double *vals, int32_t *count)
{
    #pragma omp parallel
    {
        uint64_t *cfg = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(nb + 1));
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < dim; ++r) {
            int64_t base = r * (int64_t)(nb + 1);
            int m = spin_row(states[r], nsites, nb, bi, bj, jz, jxy, hz, cfg, vals + base);
            for (int k = 0; k < m; ++k) cols[base + k] = or_rank_search(states, dim, cfg[k]);
            count[r] = m;
        }
        free(cfg);
    }
}

/* Same for the Hubbard Hamiltonian (stride 2*nh+1). */
void or_hubbard_ell(int nsites, const uint64_t *ups, int64_t dup,
                    const uint64_t *dns, int64_t ddn, int nh, const int32_t *hi,
                    const int32_t *hj, const double *ht, const double *u_site,
                    int64_t *cols, double *vals, int32_t *count)
{
    int64_t stride = 2 * (int64_t)nh + 1;
    #pragma omp parallel for schedule(static)
    for (int64_t ru = 0; ru < dup; ++ru)
        for (int64_t rd = 0; rd < ddn; ++rd) {
            int64_t r = ru * ddn + rd;
            count[r] = or_hubbard_row(nsites, ups, dup, dns, ddn, nh, hi, hj, ht,
                                      u_site, ru, rd, cols + r * stride,
                                      vals + r * stride);
        }
}

// LOBPCG for the lowest eigenpairs (HPhi update paper Sec. 3.3): subspace
// V = ({r_n}, {Phi_n}, {p_n}), H_sub = V^T H V and O_sub = V^T V, the
// generalized problem H_sub phi = E O_sub phi solved on the host, updates
// Phi = V phi, H Phi = (HV) phi, p = (r, 0, p) phi, H p = (Hr, 0, Hp) phi,
// and the point-Jacobi preconditioner r_n <- r_n / (H_xx - E_shift).
// Only the block Gram products, linear combinations, residuals and H*v run
// on the device; the (3M)-dimensional problem is solved here by cyclic
// Jacobi rotations after dropping the near-null directions of O_sub.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace hphi {
int launch_diag(hphi_ham *h, double *out, hipStream_t st);
int launch_gram(const double *const *X, int a, const double *const *Y, int b, int64_t dim, Reduce red,
                hipStream_t st);
int launch_lincomb(const double *const *V, int nin, const double *C, double *const *out, int nout, int64_t dim,
                   hipStream_t st);
int launch_resid(const double *const *HPhi, const double *const *Phi, double *const *R, int m, const double *E,
                 int estride, const double *d, double shift, int64_t dim, Reduce red, hipStream_t st);
int launch_scale_block(double *const *X, int m, const double *g, int ld, int64_t dim, hipStream_t st);

// Symmetric eigenproblem A = Q diag(w) Q^T (n x n, row-major A, overwritten),
// cyclic Jacobi; Q column j is eigenvector j; ascending order.
static void jacobi_eig(int n, std::vector<double> &A, std::vector<double> &w, std::vector<double> &Q)
{
    Q.assign((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Q[(size_t)i * n + i] = 1.0;
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    double norm = 0.0;
    for (double x : A) norm += x * x;
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += a(i, j) * a(i, j);
        if (off <= 1e-30 * norm || off == 0.0) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                if (a(p, q) == 0.0) continue;
                const double theta = (a(q, q) - a(p, p)) / (2.0 * a(p, q));
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < n; ++k) {
                    const double akp = a(k, p), akq = a(k, q);
                    a(k, p) = c * akp - s * akq;
                    a(k, q) = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    const double apk = a(p, k), aqk = a(q, k);
                    a(p, k) = c * apk - s * aqk;
                    a(q, k) = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    const double qkp = Q[(size_t)k * n + p], qkq = Q[(size_t)k * n + q];
                    Q[(size_t)k * n + p] = c * qkp - s * qkq;
                    Q[(size_t)k * n + q] = s * qkp + c * qkq;
                }
            }
    }
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return a(x, x) < a(y, y); });
    std::vector<double> Q2((size_t)n * n);
    w.resize(n);
    for (int j = 0; j < n; ++j) {
        w[j] = a(idx[j], idx[j]);
        for (int k = 0; k < n; ++k) Q2[(size_t)k * n + j] = Q[(size_t)k * n + idx[j]];
    }
    Q.swap(Q2);
}

// Lowest m solutions of H x = E O x (k x k, row-major, symmetric): returns
// false when O has fewer than m directions above the cutoff.
static bool gen_eig_lowest(int k, const std::vector<double> &H, const std::vector<double> &O, int m,
                           std::vector<double> &E, std::vector<double> &X)
{
    std::vector<double> Oc(O), s, U;
    jacobi_eig(k, Oc, s, U);
    const double smax = std::max(s.back(), 0.0);
    std::vector<int> keep;
    for (int i = 0; i < k; ++i)
        if (s[i] > 1e-10 * smax) keep.push_back(i);
    const int kk = (int)keep.size();
    if (kk < m) return false;
    // B = U_keep diag(s^-1/2) (k x kk)
    std::vector<double> B((size_t)k * kk);
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < kk; ++c) B[(size_t)r * kk + c] = U[(size_t)r * k + keep[c]] / std::sqrt(s[keep[c]]);
    // A = B^T H B
    std::vector<double> HB((size_t)k * kk, 0.0), A((size_t)kk * kk, 0.0);
    for (int r = 0; r < k; ++r)
        for (int c = 0; c < kk; ++c) {
            double acc = 0.0;
            for (int t = 0; t < k; ++t) acc += H[(size_t)r * k + t] * B[(size_t)t * kk + c];
            HB[(size_t)r * kk + c] = acc;
        }
    for (int r = 0; r < kk; ++r)
        for (int c = 0; c < kk; ++c) {
            double acc = 0.0;
            for (int t = 0; t < k; ++t) acc += B[(size_t)t * kk + r] * HB[(size_t)t * kk + c];
            A[(size_t)r * kk + c] = acc;
        }
    for (int r = 0; r < kk; ++r)
        for (int c = r + 1; c < kk; ++c) A[(size_t)r * kk + c] = A[(size_t)c * kk + r] =
                                              0.5 * (A[(size_t)r * kk + c] + A[(size_t)c * kk + r]);
    std::vector<double> w, Y;
    jacobi_eig(kk, A, w, Y);
    E.assign(w.begin(), w.begin() + m);
    X.assign((size_t)k * m, 0.0);
    for (int r = 0; r < k; ++r)
        for (int n = 0; n < m; ++n) {
            double acc = 0.0;
            for (int t = 0; t < kk; ++t) acc += B[(size_t)r * kk + t] * Y[(size_t)t * kk + n];
            X[(size_t)r * m + n] = acc;
        }
    return true;
}

// Lower bound of the spectrum from the couplings: each term's smallest
// eigenvalue, summed.
static double lower_bound(const hphi_ham *h)
{
    double lb = 0.0;
    if (h->kind == 0) {
        for (const SpinBondDev &b : h->bonds) {
            const double jz = 4.0 * b.jz4, jxy = 2.0 * b.jxy2;
            lb += std::min(jz / 4.0, -jz / 4.0 - std::fabs(jxy) / 2.0);
        }
        // field terms -h_i S^z_i: at least -|h_i| / 2 each (not stored on the host: bound by the bond sum)
    } else if (h->kind == 3) {
        // per bond |S^z S^z| <= S^2 and |S^x S^x + S^y S^y| = |S.S - S^z S^z|
        // <= S(S+1) + S^2; |S^z| <= S per field; the single-ion term at
        // min(0, d) S^2
        const double S = 0.5 * h->basis->ss.two_s;
        for (const hphi_spin_bond &b : h->sbonds)
            lb -= std::fabs(b.jz) * S * S + std::fabs(b.jxy) * (S * (S + 1.0) + S * S);
        for (double x : h->s_hz) lb -= std::fabs(x) * S;
        for (double d : h->s_dion) lb += std::min(0.0, d) * S * S;
    } else if (h->kind == 2) {
        // each bond's eigenvalues are at least -(|jx| + |jy| + |jz|) / 4, each field's -|h| / 2
        for (const hphi_xyz_bond &b : h->xyz) lb -= 0.25 * (std::fabs(b.jx) + std::fabs(b.jy) + std::fabs(b.jz));
        for (size_t i = 0; i < h->hx.size() || i < h->hz_gc.size(); ++i) {
            const double x = i < h->hx.size() ? h->hx[i] : 0.0, z = i < h->hz_gc.size() ? h->hz_gc[i] : 0.0;
            lb -= 0.5 * std::sqrt(x * x + z * z);
        }
    } else {
        for (const hphi_hop &p : h->hops) lb -= 2.0 * std::fabs(p.t);
        for (double u : h->u_site) lb += std::min(0.0, u);
        // two-body terms: n_i n_j in [0, 4], the Hund sum in [0, 2], and
        // the exchange / pair-hopping blocks at -|J| at worst
        for (const hphi_pair_term &q : h->pair_terms)
            lb += std::min(0.0, 4.0 * q.v) + std::min(0.0, -2.0 * q.j_hund) - std::fabs(q.j_ex) - std::fabs(q.j_pair);
    }
    return lb - 1e-3 * (1.0 + std::fabs(lb));
}

} // namespace hphi

using namespace hphi;

extern "C" {

int hphi_lobpcg(hphi_ham *h, const hphi_lobpcg_opts *o, double *energies_out, double *resid_out, void *vecs_dev,
                hphi_lobpcg_info *info)
{
    if (!h || !o || !energies_out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    const int M = o->n_eig;
    const int64_t dim = h->basis->dim;
    if (M < 1 || M > 32) return fail(HPHI_ERR_INVALID_ARG, "n_eig %d outside [1, 32]", M);
    if (3 * (int64_t)M > dim) return fail(HPHI_ERR_INVALID_ARG, "n_eig %d too large for dimension %lld", M, (long long)dim);
    if (o->max_iter < 1 || !(o->tol > 0.0)) return fail(HPHI_ERR_INVALID_ARG, "max_iter / tol");
    if (h->kind == 0 && h->has_field && o->precond && o->e_shift == 0.0)
        return fail(HPHI_ERR_UNSUPPORTED, "preconditioned LOBPCG with a field: give e_shift explicitly");
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)o->stream;
    HPHI_USE_HAM(h, st);
    auto t0 = std::chrono::steady_clock::now();
    const size_t vb = sizeof(double) * (size_t)dim;
    // vectors: Phi, HPhi, R, HR, P, HP and the next Phi, HPhi, P, HP
    enum { PHI, HPHI, R, HR, P, HP, PHI2, HPHI2, P2, HP2, NSET };
    DevMem store, diag, ptab, coef, gres;
    HPHI_TRY(store.alloc(vb * (size_t)M * NSET));
    std::vector<std::vector<double *>> set(NSET, std::vector<double *>(M));
    for (int s = 0; s < NSET; ++s)
        for (int n = 0; n < M; ++n) set[s][n] = store.as<double>() + ((size_t)s * M + n) * (size_t)dim;
    constexpr int kSlots = 64, kSlotLen = 96, kG = 32 * 32;
    // result slots (kG doubles each): 0 = Phi^T H Phi, 1 = R^T R, 2.. = subspace
    // blocks, kNorm = next Phi / p norms, kRes = residual norms
    constexpr int kSub = 2, kNorm = 20, kRes = 22, kNres = 23;
    HPHI_TRY(ptab.alloc(sizeof(double *) * kSlots * kSlotLen));
    HPHI_TRY(coef.alloc(sizeof(double) * 2 * 96 * 32));
    HPHI_TRY(gres.alloc(sizeof(double) * kG * kNres));
    const bool pre = o->precond != 0;
    if (pre) {
        HPHI_TRY(diag.alloc(vb));
        HPHI_TRY(launch_diag(h, diag.as<double>(), st));
    }
    const double eshift = pre ? (o->e_shift != 0.0 ? o->e_shift : lower_bound(h)) : 0.0;
    double **dptr = static_cast<double **>(ptab.p);
    double *G0 = gres.as<double>();
    // pointer tables: each launch of a phase gets its own slot; the host
    // arrays they are copied from live until the next synchronization
    int slot = 0;
    auto put = [&](const std::vector<double *> &v) -> double ** {
        double **d = dptr + (size_t)(slot++ % kSlots) * kSlotLen;
        (void)hipMemcpyAsync(d, v.data(), sizeof(double *) * v.size(), hipMemcpyHostToDevice, st);
        return d;
    };
    auto gram = [&](const std::vector<double *> &X, const std::vector<double *> &Y, int res) -> int {
        double **dx = put(X), **dy = put(Y);
        return launch_gram(dx, (int)X.size(), dy, (int)Y.size(), dim, reduce_at(h, G0 + (size_t)res * kG), st);
    };
    auto scale = [&](const std::vector<double *> &X, int res) -> int {
        return launch_scale_block(put(X), M, G0 + (size_t)res * kG, M, dim, st);
    };
    int64_t hv_calls = 0;
    auto hmult = [&](const std::vector<double *> &in, const std::vector<double *> &out) -> int {
        for (int n = 0; n < M; ++n) {
            MultArgs a{};
            a.dtype = HPHI_F64;
            a.nvec = 1;
            a.v = in[n];
            a.w = out[n];
            a.red = reduce_at(h, h->red_result.as<double>());
            a.stream = st;
            HPHI_TRY(launch_mult(h, a));
            ++hv_calls;
        }
        return HPHI_OK;
    };
    std::vector<double> Gh((size_t)kG * kNres);
    // start block: SplitMix64 uniform vectors (seed + n), normalized
    for (int n = 0; n < M; ++n) HPHI_TRY(launch_rng_uniform(HPHI_F64, set[PHI][n], dim, o->seed + (uint64_t)n, st));
    HPHI_TRY(gram(set[PHI], set[PHI], kNorm));
    HPHI_TRY(scale(set[PHI], kNorm));
    HPHI_TRY(hmult(set[PHI], set[HPHI]));
    std::vector<double> E(M, 0.0), res(M, 0.0), Ch(2 * 96 * 32);
    std::vector<double *> V, HV;
    const int blocks[3] = {R, PHI, P}, hblocks[3] = {HR, HPHI, HP};
    bool have_p = false, converged = false;
    int it = 0;
    for (; it < o->max_iter; ++it) {
        // Rayleigh quotients (Phi normalized) on the device, residuals,
        // normalized (preconditioned) residuals and H r
        HPHI_TRY(gram(set[PHI], set[HPHI], 0));
        HPHI_TRY(launch_resid(put(set[HPHI]), put(set[PHI]), put(set[R]), M, G0, M + 1,
                              pre ? diag.as<double>() : nullptr, eshift, dim,
                              reduce_at(h, G0 + (size_t)kRes * kG), st));
        HPHI_TRY(gram(set[R], set[R], 1));
        HPHI_TRY(scale(set[R], 1));
        HPHI_TRY(hmult(set[R], set[HR]));
        // subspace matrices over the blocks (R, Phi, P)
        const int nb = have_p ? 3 : 2;
        const int k = nb * M;
        int q = kSub;
        for (int bi = 0; bi < nb; ++bi)
            for (int bj = 0; bj < nb; ++bj) {
                HPHI_TRY(gram(set[blocks[bi]], set[hblocks[bj]], q++));
                if (bj >= bi) HPHI_TRY(gram(set[blocks[bi]], set[blocks[bj]], q++));
            }
        // one synchronization per iteration: all small results at once
        HPHI_HIP(hipMemcpyAsync(Gh.data(), G0, sizeof(double) * Gh.size(), hipMemcpyDeviceToHost, st));
        HPHI_HIP(hipStreamSynchronize(st));
        slot = 0;
        double worst = 0.0;
        for (int n = 0; n < M; ++n) {
            E[n] = Gh[(size_t)n * (M + 1)];
            res[n] = std::sqrt(std::max(Gh[(size_t)kRes * kG + n], 0.0));
            worst = std::max(worst, res[n]);
        }
        if (worst < o->tol) {
            converged = true;
            break;
        }
        std::vector<double> Hs((size_t)k * k), Os((size_t)k * k);
        q = kSub;
        for (int bi = 0; bi < nb; ++bi)
            for (int bj = 0; bj < nb; ++bj) {
                const double *gh = Gh.data() + (size_t)(q++) * kG;
                for (int i = 0; i < M; ++i)
                    for (int j = 0; j < M; ++j) Hs[(size_t)(bi * M + i) * k + bj * M + j] = gh[(size_t)i * M + j];
                if (bj < bi) continue;
                const double *go = Gh.data() + (size_t)(q++) * kG;
                for (int i = 0; i < M; ++i)
                    for (int j = 0; j < M; ++j) {
                        Os[(size_t)(bi * M + i) * k + bj * M + j] = go[(size_t)i * M + j];
                        Os[(size_t)(bj * M + j) * k + bi * M + i] = go[(size_t)i * M + j];
                    }
            }
        for (int i = 0; i < k; ++i)
            for (int j = i + 1; j < k; ++j) Hs[(size_t)i * k + j] = Hs[(size_t)j * k + i] =
                                                0.5 * (Hs[(size_t)i * k + j] + Hs[(size_t)j * k + i]);
        std::vector<double> En, X;
        if (!gen_eig_lowest(k, Hs, Os, M, En, X)) {
            if (!have_p) return fail(HPHI_ERR_UNSUPPORTED, "LOBPCG subspace lost rank");
            have_p = false;   // restart without the conjugate directions
            continue;
        }
        // updates: Phi = V X, HPhi = HV X, p = (r, 0, p) X, Hp = (Hr, 0, Hp) X
        V.clear();
        HV.clear();
        for (int bi = 0; bi < nb; ++bi) {
            V.insert(V.end(), set[blocks[bi]].begin(), set[blocks[bi]].end());
            HV.insert(HV.end(), set[hblocks[bi]].begin(), set[hblocks[bi]].end());
        }
        std::copy(X.begin(), X.end(), Ch.begin());
        std::copy(X.begin(), X.end(), Ch.begin() + 96 * 32);
        for (int i = M; i < 2 * M; ++i)
            for (int n = 0; n < M; ++n) Ch[96 * 32 + (size_t)i * M + n] = 0.0;
        HPHI_HIP(hipMemcpyAsync(coef.p, Ch.data(), sizeof(double) * Ch.size(), hipMemcpyHostToDevice, st));
        const double *cx = coef.as<double>(), *cp = coef.as<double>() + 96 * 32;
        HPHI_TRY(launch_lincomb(put(V), k, cx, put(set[PHI2]), M, dim, st));
        HPHI_TRY(launch_lincomb(put(HV), k, cx, put(set[HPHI2]), M, dim, st));
        HPHI_TRY(launch_lincomb(put(V), k, cp, put(set[P2]), M, dim, st));
        HPHI_TRY(launch_lincomb(put(HV), k, cp, put(set[HP2]), M, dim, st));
        // normalize Phi (H Phi alike) and p (H p alike) from their Gram diagonals
        HPHI_TRY(gram(set[PHI2], set[PHI2], kNorm));
        HPHI_TRY(scale(set[PHI2], kNorm));
        HPHI_TRY(scale(set[HPHI2], kNorm));
        HPHI_TRY(gram(set[P2], set[P2], kNorm + 1));
        HPHI_TRY(scale(set[P2], kNorm + 1));
        HPHI_TRY(scale(set[HP2], kNorm + 1));
        std::swap(set[PHI], set[PHI2]);
        std::swap(set[HPHI], set[HPHI2]);
        std::swap(set[P], set[P2]);
        std::swap(set[HP], set[HP2]);
        have_p = true;
    }
    for (int n = 0; n < M; ++n) {
        energies_out[n] = E[n];
        if (resid_out) resid_out[n] = res[n];
    }
    if (vecs_dev)
        for (int n = 0; n < M; ++n)
            HPHI_HIP(hipMemcpyAsync(static_cast<double *>(vecs_dev) + (size_t)n * dim, set[PHI][n], vb,
                                    hipMemcpyDeviceToDevice, st));
    HPHI_HIP(hipStreamSynchronize(st));
    if (info) {
        info->iterations = it;
        info->converged = converged ? 1 : 0;
        info->hv_calls = hv_calls;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return HPHI_OK;
}

} // extern "C"

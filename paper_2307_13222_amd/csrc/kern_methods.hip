// Kernels of the cTPQ and shifted-COCG drivers.
//
// Shifted COCG (conjugate orthogonal CG for complex symmetric systems, van
// der Vorst and Melissen 1990; shifted form: Frommer 2003, Takayama et al.
// 2006), used for D(z) = <b|(z - H)^-1|b> (HPhi update paper Sec. 3.2,
// method "CG"). Seed system A = z_s - H (complex symmetric since H is real
// symmetric), bilinear products u^T v without conjugation:
//   p_k = r_k + beta_{k-1} p_{k-1};  alpha_k = r_k^T r_k / p_k^T A p_k;
//   r_{k+1} = r_k - alpha_k A p_k;   beta_k = r_{k+1}^T r_{k+1} / r_k^T r_k.
// Each shifted system (A + sigma) x = b, sigma = z_j - z_s, has a collinear
// residual r_k / pi_k with pi_k = R_k(-sigma) for the seed residual
// polynomial R_k:
//   pi_{k+1} = (1 + alpha_k beta_{k-1} / alpha_{k-1} + alpha_k sigma) pi_k
//              - (alpha_k beta_{k-1} / alpha_{k-1}) pi_{k-1},
//   alpha^s = (pi_k / pi_{k+1}) alpha_k,  beta^s = (pi_k / pi_{k+1})^2 beta_k.
// Only the projections X = b^H x^s and P = b^H p^s are carried:
//   X += alpha^s P;  P = (b^H r_{k+1}) / pi_{k+1} + beta^s P.
#include "kern_common.h"

namespace hphi {


// init: rho = b^T b, |b|^2; r = p = b; shift state.
__global__ __launch_bounds__(kBlock) void k_cocg_init(const double *b, double *r, double *p, int64_t dim,
                                                      CgDev *cg, ShiftDev *sh, int nsh, double tol, Reduce red)
{
    __shared__ double shr[kBlock / kWave * 4];
    __shared__ double blk[4];
    double a[3] = {0, 0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double br = b[2 * i], bi = b[2 * i + 1];
        r[2 * i] = br; r[2 * i + 1] = bi;
        p[2 * i] = br; p[2 * i + 1] = bi;
        a[0] += br * br - bi * bi;
        a[1] += 2 * br * bi;
        a[2] += br * br + bi * bi;
    }
    block_sum<3>(a, shr);
    if (threadIdx.x == 0) { blk[0] = a[0]; blk[1] = a[1]; blk[2] = a[2]; }
    __syncthreads();
    if (grid_finish(blk, 3, red, shr)) {
        __syncthreads();
        const double bn2 = red.result[2];
        for (int j = threadIdx.x; j < nsh; j += blockDim.x) {
            sh[j].pi = {1.0, 0.0};
            sh[j].pi_prev = {1.0, 0.0};
            sh[j].X = {0.0, 0.0};
            sh[j].P = {bn2, 0.0};
            sh[j].res = 1.0;
            sh[j].conv = 0;
        }
        if (threadIdx.x == 0) {
            cg->rho = {red.result[0], red.result[1]};
            cg->bnorm2 = bn2;
            cg->alpha = {1.0, 0.0};   // plays alpha_{-1}
            cg->beta = {0.0, 0.0};    // plays beta_{-1}
            cg->iter = 0;
            cg->breakdown = 0;
            cg->max_res = 1.0;
        }
        (void)tol;
        __threadfence();
    }
}

// The streaming COCG kernels keep four independent elements (16 B each) in
// flight per thread and trip; the tail loop takes the rest.

// mu = p^T (z_s p - h) with h = H p; alpha_k = rho / mu.
__global__ __launch_bounds__(kBlock) void k_cocg_mu(const double *p, const double *h, int64_t dim, CgDev *cg,
                                                    Reduce red)
{
    __shared__ double shr[kBlock / kWave * 4];
    __shared__ double blk[4];
    const cd zs = cg->zs;
    const double2 *P = reinterpret_cast<const double2 *>(p);
    const double2 *H = reinterpret_cast<const double2 *>(h);
    double a[2] = {0, 0};
    auto add = [&](double2 pp, double2 hh) {
        const cd pv = {pp.x, pp.y};
        const cd ap = csub(cmul(zs, pv), cd{hh.x, hh.y});
        const cd t = cmul(pv, ap);
        a[0] += t.re;
        a[1] += t.im;
    };
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * st < dim; i += 4 * st) {
        double2 pv[4], hv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pv[u] = P[i + u * st];
            hv[u] = H[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) add(pv[u], hv[u]);
    }
    for (; i < dim; i += st) add(P[i], H[i]);
    block_sum<2>(a, shr);
    if (threadIdx.x == 0) { blk[0] = a[0]; blk[1] = a[1]; }
    __syncthreads();
    if (grid_finish(blk, 2, red, shr) && threadIdx.x == 0) cocg_alpha_step(cg, {red.result[0], red.result[1]});
}

// Per-shift scalar recurrences (the threads of one block, one shift each at
// a time) and the max residual over the unconverged shifts.
__device__ void cocg_shifts_step(CgDev *cg, ShiftDev *sh, int nsh, double tol, double *smax)
{
    const cd al = cg->alpha, be = cg->beta, alp = cg->alpha_prev, bep = cg->beta_prev;
    const cd bhr = cg->bhr;
    const double rn = sqrt(cg->rnorm2), bn = sqrt(cg->bnorm2);
    const cd ratio = cabs2(alp) > 0.0 ? cdiv(cmul(al, bep), alp) : cd{0.0, 0.0};
    double mx = 0.0;
    for (int j = threadIdx.x; j < nsh; j += blockDim.x) {
        ShiftDev s = sh[j];
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
            if (s.res < tol) s.conv = 1;
            sh[j] = s;
        }
        mx = fmax(mx, s.conv ? 0.0 : s.res);
    }
    smax[threadIdx.x] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int t = 0; t < (int)blockDim.x; ++t) m = fmax(m, smax[t]);
        cg->max_res = m;
        __threadfence();
    }
}

// r -= alpha (z_s p - h); rho' = r^T r, |r|^2, b^H r; beta = rho'/rho; then
// (last block) the per-shift recurrences.
__global__ __launch_bounds__(kBlock) void k_cocg_r(double *r, const double *p, const double *h, const double *b,
                                                   int64_t dim, CgDev *cg, ShiftDev *sh, int nsh, double tol,
                                                   Reduce red)
{
    __shared__ double shr[kBlock / kWave * 8];
    __shared__ double blk[8];
    __shared__ double smax[kBlock];
    const cd zs = cg->zs, al = cg->alpha;
    const double2 *P = reinterpret_cast<const double2 *>(p);
    const double2 *H = reinterpret_cast<const double2 *>(h);
    const double2 *B = reinterpret_cast<const double2 *>(b);
    double2 *R = reinterpret_cast<double2 *>(r);
    double a[5] = {0, 0, 0, 0, 0};
    auto step = [&](int64_t k, double2 pp, double2 hh, double2 rr, double2 bb) {
        const cd ap = csub(cmul(zs, cd{pp.x, pp.y}), cd{hh.x, hh.y});
        const cd rv = csub(cd{rr.x, rr.y}, cmul(al, ap));
        R[k] = make_double2(rv.re, rv.im);
        a[0] += rv.re * rv.re - rv.im * rv.im;
        a[1] += 2 * rv.re * rv.im;
        a[2] += rv.re * rv.re + rv.im * rv.im;
        a[3] += bb.x * rv.re + bb.y * rv.im;      // conj(b) r
        a[4] += bb.x * rv.im - bb.y * rv.re;
    };
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * st < dim; i += 4 * st) {
        double2 pv[4], hv[4], rv[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            pv[u] = P[i + u * st];
            hv[u] = H[i + u * st];
            rv[u] = R[i + u * st];
            bv[u] = B[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) step(i + u * st, pv[u], hv[u], rv[u], bv[u]);
    }
    for (; i < dim; i += st) step(i, P[i], H[i], R[i], B[i]);
    block_sum<5>(a, shr);
    if (threadIdx.x == 0)
        for (int t = 0; t < 5; ++t) blk[t] = a[t];
    __syncthreads();
    if (!grid_finish(blk, 5, red, shr)) return;
    if (threadIdx.x == 0) {
        const cd rho1 = {red.result[0], red.result[1]};
        cg->rnorm2 = red.result[2];
        cg->bhr = {red.result[3], red.result[4]};
        if (cabs2(cg->rho) == 0.0) {
            cg->breakdown = 1;
            cg->beta = {0.0, 0.0};
        } else {
            cg->beta = cdiv(rho1, cg->rho);
        }
        cg->rho = rho1;
        cg->iter += 1;
        __threadfence();
    }
    __syncthreads();
    cocg_shifts_step(cg, sh, nsh, tol, smax);
}

// p = r + beta p
__global__ __launch_bounds__(kBlock) void k_cocg_p(const double *r, double *p, int64_t dim, const CgDev *cg)
{
    const cd be = cg->beta;
    const double2 *R = reinterpret_cast<const double2 *>(r);
    double2 *P = reinterpret_cast<double2 *>(p);
    auto step = [&](int64_t k, double2 rr, double2 pp) {
        const cd t = cmul(be, cd{pp.x, pp.y});
        P[k] = make_double2(rr.x + t.re, rr.y + t.im);
    };
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + 3 * st < dim; i += 4 * st) {
        double2 rv[4], pv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            rv[u] = R[i + u * st];
            pv[u] = P[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) step(i + u * st, rv[u], pv[u]);
    }
    for (; i < dim; i += st) step(i, R[i], P[i]);
}

static int gridn(int64_t n)
{
    int64_t g = (n + kBlock * 2 - 1) / (kBlock * 2);
    return (int)(g < 1 ? 1 : (g > 2048 ? 2048 : g));
}

int launch_cocg_init(const void *b, void *r, void *p, int64_t dim, void *cg, void *sh, int nsh, double tol,
                     Reduce red, hipStream_t st)
{
    hipLaunchKernelGGL(k_cocg_init, dim3(gridn(dim)), dim3(kBlock), 0, st, (const double *)b, (double *)r,
                       (double *)p, dim, (CgDev *)cg, (ShiftDev *)sh, nsh, tol, red);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

int launch_cocg_iter(void *r, void *p, const void *h, const void *b, int64_t dim, void *cg, void *sh,
                     int nsh, double tol, Reduce red, hipStream_t st, bool mu_done)
{
    // at least 8 elements per thread, so the four-element trips dominate
    int64_t g8 = (dim + kBlock * 8 - 1) / (kBlock * 8);
    const int g = (int)(g8 < 1 ? 1 : (g8 > 2048 ? 2048 : g8));
    // (mu_done: the product's epilogue already formed mu and alpha)
    if (!mu_done)
        hipLaunchKernelGGL(k_cocg_mu, dim3(g), dim3(kBlock), 0, st, (const double *)p, (const double *)h,
                           dim, (CgDev *)cg, red);
    hipLaunchKernelGGL(k_cocg_r, dim3(g), dim3(kBlock), 0, st, (double *)r, (const double *)p,
                       (const double *)h, (const double *)b, dim, (CgDev *)cg, (ShiftDev *)sh, nsh, tol, red);
    hipLaunchKernelGGL(k_cocg_p, dim3(g), dim3(kBlock), 0, st, (const double *)r, (double *)p, dim,
                       (const CgDev *)cg);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// out = (Re b, 0) for part 0, (Im b, 0) for part 1 (complex vectors).
__global__ void k_cplx_part(const double *b, double *out, int64_t dim, int part)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim;
         i += (int64_t)gridDim.x * blockDim.x) {
        out[2 * i] = b[2 * i + part];
        out[2 * i + 1] = 0.0;
    }
}

int launch_cplx_part(const void *b, void *out, int64_t dim, int part, hipStream_t st)
{
    hipLaunchKernelGGL(k_cplx_part, dim3(gridn(dim)), dim3(kBlock), 0, st, (const double *)b, (double *)out,
                       dim, part);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

// s[l] = 1/sqrt(n[2*(l/2)] + n[2*(l/2)+1]) for nl lanes (complex pairs).
__global__ void k_pair_rsqrt(const double *n, double *s, int nl)
{
    const int l = threadIdx.x;
    if (l < nl) s[l] = 1.0 / sqrt(n[2 * (l / 2)] + n[2 * (l / 2) + 1]);
}

int launch_pair_rsqrt(const double *n, double *s, int nl, hipStream_t st)
{
    hipLaunchKernelGGL(k_pair_rsqrt, dim3(1), dim3(64), 0, st, n, s, nl);
    HPHI_HIP(hipGetLastError());
    return HPHI_OK;
}

} // namespace hphi

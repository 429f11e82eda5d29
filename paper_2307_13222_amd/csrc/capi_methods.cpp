// C ABI of the methods built on H*v: cTPQ (block Taylor propagator) and the
// dynamical correlation function by shifted COCG.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

using namespace hphi;

namespace {



} // namespace

extern "C" {

// cTPQ. The propagator U_c = sum_{n<=n_max} x^n / n!, x = -dtau H / 2, is
// evaluated by Horner's rule y <- phi + (x / n) y for n = n_max .. 1 (the
// same polynomial as the term-by-term sum), one block H*V per order with the
// epilogue w = c1 H y + c2 phi fused into the kernel. The first order of each
// step applies H to the normalized state itself, so its raw FP64 dots give
// <phi|H|phi> and |H phi|^2 at beta_{k-1}; a streaming pass over the last
// order's stored output gives the squared norm N_k = D_k of U_c phi.
int hphi_ctpq(hphi_ham *h, const hphi_ctpq_opts *o, void *phi_dev, double *D_out, double *E_out,
              double *E2_out)
{
    if (!h || !o || !phi_dev) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (o->n_vec < 1 || o->n_vec > 16) return fail(HPHI_ERR_INVALID_ARG, "n_vec %d outside [1, 16]", o->n_vec);
    if (o->n_max < 1 || o->n_max > 64) return fail(HPHI_ERR_INVALID_ARG, "n_max %d outside [1, 64]", o->n_max);
    if (o->k_steps < 0 || !(o->dtau > 0.0)) return fail(HPHI_ERR_INVALID_ARG, "k_steps / dtau");
    if (o->storage != HPHI_C128 && o->storage != HPHI_C64)
        return fail(HPHI_ERR_INVALID_ARG, "cTPQ storage must be C128 or C64");
    if (h->kind != 0 && o->n_vec != 1)
        return fail(HPHI_ERR_UNSUPPORTED, "Hubbard and SpinGC cTPQ run one vector per call");
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)o->stream;
    HPHI_USE_HAM(h, st);
    // the legacy default stream cannot be captured: a stream of our own,
    // after the work queued on the default one
    OwnStream own;
    if (o->use_graph && !st) HPHI_TRY(own.make(&st));
    const int dt = o->storage, nv = o->n_vec, nl = 2 * nv;
    const int64_t dim = h->basis->dim;
    const size_t bytes = (size_t)dim * nl * dtype_size(dt);
    DevMem y1, y2, yraw, scal, res_first, res_last;
    HPHI_TRY(y1.alloc(bytes));
    HPHI_TRY(y2.alloc(bytes));
    // wide spin blocks: the first order stores H phi itself and a streaming
    // pass takes <phi|H phi>, |H phi|^2 from it (the same FP32/FP64 values
    // the fused dots would use; the block kernel with 2 x nl FP64 dot
    // accumulators per thread runs far fewer waves)
    // (on the implicit basis the block-staged product, the one there for
    // several lanes, has no fused dots: the same streaming pass)
    const bool raw_dots = h->kind == 0 && ((nl >= 8 && spin_stored_path(h)) ||
                                           (!spin_stored_path(h) && spin_split_mode(h, true) == 2));
    if (raw_dots) HPHI_TRY(yraw.alloc(bytes));
    HPHI_TRY(scal.alloc(sizeof(double) * (2 * (size_t)o->n_max + 2 + 64)));
    HPHI_TRY(res_first.alloc(sizeof(double) * 2 * 64));
    HPHI_TRY(res_last.alloc(sizeof(double) * 2 * 64));
    // epilogue coefficients: order n uses (c1, c2) = (-dtau / (2 n), 1)
    std::vector<double> cf(2 * (size_t)o->n_max + 2, 0.0);
    for (int n = 1; n <= o->n_max; ++n) {
        cf[2 * n] = -o->dtau / (2.0 * n);
        cf[2 * n + 1] = 1.0;
    }
    HPHI_HIP(hipMemcpyAsync(scal.p, cf.data(), sizeof(double) * cf.size(), hipMemcpyHostToDevice, st));
    HPHI_HIP(hipStreamSynchronize(st));
    double *d_coef = scal.as<double>();
    double *d_lane_scale = d_coef + 2 * o->n_max + 2;

    void *A = phi_dev;
    if (o->phi0_dev) HPHI_HIP(hipMemcpyAsync(A, o->phi0_dev, bytes, hipMemcpyDeviceToDevice, st));
    else HPHI_TRY(launch_rng_cgauss(dt, A, dim, nv, o->seed, st));

    std::vector<double> hl(2 * nl);
    // N_0 and normalization
    HPHI_TRY(launch_dots(dt, nl, dim, A, A, reduce_at(h, res_last.as<double>()), 1, st));
    HPHI_HIP(hipMemcpyAsync(hl.data(), res_last.p, sizeof(double) * nl, hipMemcpyDeviceToHost, st));
    HPHI_TRY(launch_pair_rsqrt(res_last.as<double>(), d_lane_scale, nl, st));
    HPHI_TRY(launch_scale_lanes(dt, nl, dim, A, d_lane_scale, 0, st));
    HPHI_HIP(hipStreamSynchronize(st));
    for (int j = 0; j < nv; ++j)
        if (D_out) D_out[j] = hl[2 * j] + hl[2 * j + 1];

    void *Y[2] = {y1.p, y2.p};
    const int K = o->k_steps;
    // Per-step results stay on the device (row k of `stage`: <H> and <H^2>
    // lanes, then the new squared norms) and come back once at the end, so a
    // step needs no host round trip and its launches can be replayed from a
    // graph. `step` enqueues step k (k < K: the whole propagator; k == K:
    // only the first-order product).
    const int row = 3 * nl;
    DevMem stage, counter;
    HPHI_TRY(stage.alloc(sizeof(double) * (size_t)row * (K + 1)));
    HPHI_TRY(counter.alloc(sizeof(int) * 2));
    HPHI_TRY(launch_zero(counter.p, sizeof(int) * 2, st));
    auto step = [&](bool last_step) -> int {
        const void *src = A;
        int yb = 0;
        for (int n = o->n_max; n >= 1; --n) {
            const bool first = (n == o->n_max);
            MultArgs a{};
            a.dtype = dt;
            a.nvec = nv;
            a.v = src;
            a.w = Y[yb];
            a.u = A;
            a.coef = d_coef + 2 * n;
            a.stream = st;
            if (first && !raw_dots) {
                a.dots = 1;
                a.dot_raw = 1;
                a.red = reduce_at(h, res_first.as<double>());
            } else {
                a.red = reduce_at(h, h->red_result.as<double>());
                if (first) a.raw_out = yraw.p;
            }
            HPHI_TRY(launch_mult(h, a));
            if (first && raw_dots)
                HPHI_TRY(launch_dots_xy_yy(dt, nl, dim, src, yraw.p, reduce_at(h, res_first.as<double>()), st));
            if (last_step) break;
            src = Y[yb];
            yb ^= 1;
        }
        HPHI_TRY(launch_record(res_first.as<double>(), 2 * nl, stage.as<double>(), row, counter.as<int>(), 0, st));
        if (!last_step) {
            // the last order wrote Y[yb ^ 1]; its lanes' |.|^2 from one
            // streaming pass over the stored values (the fused dots of the
            // wide block kernel cost more registers than this pass costs)
            void *out = Y[yb ^ 1];
            double *nrm = res_last.as<double>();
            HPHI_TRY(launch_dots_xy_yy(dt, nl, dim, out, out, reduce_at(h, nrm), st));
            HPHI_TRY(launch_record(nrm, nl, stage.as<double>() + 2 * nl, row, counter.as<int>(), 1, st));
            HPHI_TRY(launch_pair_rsqrt(nrm, d_lane_scale, nl, st));
            HPHI_TRY(launch_scale_lanes(dt, nl, dim, out, d_lane_scale, 0, st));
            // new state: copy back into the caller's buffer
            HPHI_HIP(hipMemcpyAsync(A, out, bytes, hipMemcpyDeviceToDevice, st));
        }
        return HPHI_OK;
    };
    int k = 0;
    if (o->use_graph && K >= 2) {
        // one step captured and replayed: the same launches on the same
        // buffers, so the same numbers as the eager steps
        HPHI_TRY(step(false));
        ++k;
        hipGraph_t gph = nullptr;
        hipGraphExec_t exec = nullptr;
        HPHI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = step(false);
        const hipError_t e = hipStreamEndCapture(st, &gph);
        if (rc != HPHI_OK) {
            if (gph) (void)hipGraphDestroy(gph);
            return rc;
        }
        if (e != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gph);
        if (ei != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
        hipError_t el = hipSuccess;
        for (; k < K && el == hipSuccess; ++k) el = hipGraphLaunch(exec, st);
        (void)hipGraphExecDestroy(exec);
        if (el != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph launch: %s", hipGetErrorString(el));
    }
    for (; k < K; ++k) HPHI_TRY(step(false));
    HPHI_TRY(step(true));
    std::vector<double> hs((size_t)row * (K + 1));
    HPHI_HIP(hipMemcpyAsync(hs.data(), stage.p, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    for (int kk = 0; kk <= K; ++kk) {
        const double *hf = hs.data() + (size_t)kk * row, *hl2 = hf + 2 * nl;
        for (int j = 0; j < nv; ++j) {
            if (E_out) E_out[(size_t)kk * nv + j] = hf[2 * j] + hf[2 * j + 1];
            if (E2_out) E2_out[(size_t)kk * nv + j] = hf[nl + 2 * j] + hf[nl + 2 * j + 1];
            if (kk < K && D_out) D_out[(size_t)(kk + 1) * nv + j] = hl2[2 * j] + hl2[2 * j + 1];
        }
    }
    return HPHI_OK;
}

int hphi_time_evolve(hphi_ham *h, const hphi_tevol_opts *o, void *psi_dev, double *norm_out, double *energy_out,
                     double *docc_out)
{
    if (!h || !o || !psi_dev) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (o->n_vec < 1 || o->n_vec > 16) return fail(HPHI_ERR_INVALID_ARG, "n_vec %d outside [1, 16]", o->n_vec);
    if (o->n_max < 1 || o->n_max > 64) return fail(HPHI_ERR_INVALID_ARG, "n_max %d outside [1, 64]", o->n_max);
    if (o->n_steps < 0 || !std::isfinite(o->dt) || o->dt == 0.0)
        return fail(HPHI_ERR_INVALID_ARG, "n_steps / dt");
    if (o->storage != HPHI_C128 && o->storage != HPHI_C64)
        return fail(HPHI_ERR_INVALID_ARG, "time evolution storage must be C128 or C64");
    if (h->kind != 0 && o->n_vec != 1)
        return fail(HPHI_ERR_UNSUPPORTED, "Hubbard and SpinGC time evolution run one vector per call");
    if (docc_out && h->kind != 1) return fail(HPHI_ERR_INVALID_ARG, "double occupancy needs a Hubbard model");
    if (o->first_frame < 0 || o->first_frame >= (h->td ? h->td->n : 1))
        return fail(HPHI_ERR_INVALID_ARG, "first_frame %d outside the Hamiltonian's frames", o->first_frame);
    if (h->td && o->use_graph)
        return fail(HPHI_ERR_UNSUPPORTED, "frames change the products' launch arguments between steps: no graph replay");
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)o->stream;
    HPHI_USE_HAM(h, st);
    OwnStream own;
    if (o->use_graph && !st) HPHI_TRY(own.make(&st));
    const int dt = o->storage, nv = o->n_vec, nl = 2 * nv;
    const int64_t dim = h->basis->dim;
    const size_t bytes = (size_t)dim * nl * dtype_size(dt);
    DevMem y1, y2, yraw, scal, res_e, res_n, res_d;
    HPHI_TRY(y1.alloc(bytes));
    HPHI_TRY(y2.alloc(bytes));
    // spin sectors on the implicit basis run the block-staged product, which
    // has no fused dots: <psi|H psi> from its raw output by a streaming pass
    const bool raw_e = h->kind == 0 && !spin_stored_path(h) && spin_split_mode(h, true) == 2;
    if (raw_e) HPHI_TRY(yraw.alloc(bytes));
    HPHI_TRY(scal.alloc(sizeof(double) * 4 * ((size_t)o->n_max + 1)));
    HPHI_TRY(res_e.alloc(sizeof(double) * 2 * 64));
    HPHI_TRY(res_n.alloc(sizeof(double) * 2 * 64));
    HPHI_TRY(res_d.alloc(sizeof(double) * 8));
    // Horner order n: y <- psi + (-i dt / n) H y, i.e. c1 = -i dt / n, c2 = 1
    std::vector<double> cf(4 * ((size_t)o->n_max + 1), 0.0);
    for (int n = 1; n <= o->n_max; ++n) {
        cf[4 * n + 0] = 0.0;
        cf[4 * n + 1] = 1.0;
        cf[4 * n + 2] = -o->dt / n;
        cf[4 * n + 3] = 0.0;
    }
    HPHI_HIP(hipMemcpyAsync(scal.p, cf.data(), sizeof(double) * cf.size(), hipMemcpyHostToDevice, st));
    HPHI_HIP(hipStreamSynchronize(st));
    const double *d_coef = scal.as<double>();
    void *A = psi_dev;
    void *Y[2] = {y1.p, y2.p};
    const int K = o->n_steps;
    // Per recorded time, on the device (row k of `stage`: <psi|H|psi>
    // lanes, <psi|psi> lanes, double occupancy), copied back once at the
    // end; `step` enqueues time k (k < K: observables and one Taylor step;
    // k == K: observables only), so steps replay from a graph.
    const int row = 2 * nl + 1;
    DevMem stage, counter;
    HPHI_TRY(stage.alloc(sizeof(double) * (size_t)row * (K + 1)));
    HPHI_TRY(counter.alloc(sizeof(int) * 4));
    HPHI_TRY(launch_zero(counter.p, sizeof(int) * 4, st));
    HPHI_TRY(launch_zero(res_d.p, sizeof(double) * 8, st));
    // time t_kk: with frames, H(t_kk) is frame min(first_frame + kk,
    // n_frames - 1), held over the step to t_kk+1
    auto step = [&](int kk, bool last_step) -> int {
        if (h->td) HPHI_TRY(ham_apply_frame(h, (int)std::min<int64_t>((int64_t)o->first_frame + kk, h->td->n - 1), st));
        HPHI_TRY(launch_dots(dt, nl, dim, A, A, reduce_at(h, res_n.as<double>()), 1, st));
        if (docc_out) HPHI_TRY(launch_docc(h, dt, A, reduce_at(h, res_d.as<double>()), st));
        if (last_step) {
            MultArgs a{};
            a.dtype = dt;
            a.nvec = nv;
            a.v = A;
            a.w = Y[0];
            a.dots = raw_e ? 0 : 1;
            a.dot_raw = 1;
            a.red = reduce_at(h, res_e.as<double>());
            a.stream = st;
            HPHI_TRY(launch_mult(h, a));
            if (raw_e) HPHI_TRY(launch_dots_xy_yy(dt, nl, dim, A, Y[0], reduce_at(h, res_e.as<double>()), st));
        } else {
            const void *src = A;
            int yb = 0;
            for (int n = o->n_max; n >= 1; --n) {
                MultArgs a{};
                a.dtype = dt;
                a.nvec = nv;
                a.v = src;
                a.w = Y[yb];
                a.u = A;
                a.coef = d_coef + 4 * n;
                a.coef_cplx = 1;
                a.stream = st;
                if (n == o->n_max && !raw_e) {
                    a.dots = 1;     // <psi, H psi> rides on the first product
                    a.dot_raw = 1;
                    a.red = reduce_at(h, res_e.as<double>());
                } else {
                    a.red = reduce_at(h, h->red_result.as<double>());
                    if (n == o->n_max) a.raw_out = yraw.p;
                }
                HPHI_TRY(launch_mult(h, a));
                if (n == o->n_max && raw_e)
                    HPHI_TRY(launch_dots_xy_yy(dt, nl, dim, A, yraw.p, reduce_at(h, res_e.as<double>()), st));
                src = Y[yb];
                yb ^= 1;
            }
        }
        HPHI_TRY(launch_record(res_e.as<double>(), nl, stage.as<double>(), row, counter.as<int>(), 0, st));
        HPHI_TRY(launch_record(res_n.as<double>(), nl, stage.as<double>() + nl, row, counter.as<int>(), 1, st));
        HPHI_TRY(launch_record(res_d.as<double>(), 1, stage.as<double>() + 2 * nl, row, counter.as<int>(), 2, st));
        if (!last_step) {
            // the order-1 product holds psi(t_{k+1}); copy it into the caller's buffer
            const void *out = (o->n_max % 2 == 1) ? Y[0] : Y[1];
            HPHI_HIP(hipMemcpyAsync(A, out, bytes, hipMemcpyDeviceToDevice, st));
        }
        return HPHI_OK;
    };
    int k = 0;
    if (o->use_graph && K >= 2) {
        HPHI_TRY(step(k, false));
        ++k;
        hipGraph_t gph = nullptr;
        hipGraphExec_t exec = nullptr;
        HPHI_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        const int rc = step(k, false);
        const hipError_t e = hipStreamEndCapture(st, &gph);
        if (rc != HPHI_OK) {
            if (gph) (void)hipGraphDestroy(gph);
            return rc;
        }
        if (e != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
        const hipError_t ei = hipGraphInstantiate(&exec, gph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gph);
        if (ei != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(ei));
        hipError_t el = hipSuccess;
        for (; k < K && el == hipSuccess; ++k) el = hipGraphLaunch(exec, st);
        (void)hipGraphExecDestroy(exec);
        if (el != hipSuccess) return fail(HPHI_ERR_DEVICE, "graph launch: %s", hipGetErrorString(el));
    }
    for (; k < K; ++k) HPHI_TRY(step(k, false));
    HPHI_TRY(step(K, true));
    std::vector<double> hs((size_t)row * (K + 1));
    HPHI_HIP(hipMemcpyAsync(hs.data(), stage.p, sizeof(double) * hs.size(), hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    for (int kk = 0; kk <= K; ++kk) {
        const double *he = hs.data() + (size_t)kk * row, *hn = he + nl;
        for (int j = 0; j < nv; ++j) {
            const double nrm = hn[2 * j] + hn[2 * j + 1];
            if (norm_out) norm_out[(size_t)kk * nv + j] = nrm;
            if (energy_out) energy_out[(size_t)kk * nv + j] = (he[2 * j] + he[2 * j + 1]) / nrm;
        }
        if (docc_out) docc_out[kk] = he[2 * nl] / (hn[0] + hn[1]) / h->basis->n_sites;
    }
    return HPHI_OK;
}

int hphi_lanczos_batch(hphi_batch_item *items, int n, void *stream)
{
    if (!items || n < 1) return fail(HPHI_ERR_INVALID_ARG, "empty batch");
    for (int i = 0; i < n; ++i) {
        if (!items[i].ham) return fail(HPHI_ERR_INVALID_ARG, "item %d has no Hamiltonian", i);
        if (items[i].max_iter < 1 || items[i].max_iter > 100000)
            return fail(HPHI_ERR_INVALID_ARG, "item %d max_iter %d", i, items[i].max_iter);
        if (items[i].ham->basis->ctx != items[0].ham->basis->ctx)
            return fail(HPHI_ERR_INVALID_ARG, "batch items on different contexts");
    }
    DeviceGuard g(items[0].ham->basis->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // Team shape of each request (from its dimension alone). Requests whose
    // vector fits in LDS run on one workgroup each (throughput) unless the
    // whole launch fits on the CUs as teams (one workgroup per CU), which
    // then cut the latency (16-site requests, 13 members each: 19 requests
    // as teams 5.3 ms, on one workgroup each 9.7 ms). The other requests always run as teams, in launches of
    // at most one workgroup per CU so that all members of a launch are
    // resident together. The reductions are ordered by rows, so every way
    // gives the same numbers.
    const size_t kLdsCap = 150 * 1024;
    std::vector<size_t> q_off(n), ab_off(n), part_off(n);
    std::vector<int> tw(n), tbase(n);
    std::vector<char> lds_ok(n);
    size_t nq = 0, nab = 0, npart = 0;
    int team_total = 0, team_max = 1;
    for (int i = 0; i < n; ++i) {
        const Species &s = items[i].ham->basis->sp[0];
        q_off[i] = nq;
        ab_off[i] = nab;
        part_off[i] = npart;
        nq += 3 * (size_t)s.dim;
        nab += 2 * (size_t)items[i].max_iter + 1;
        npart += batch_part_doubles(s.dim);
        int rows = 0;
        batch_team_shape(s.dim, &tw[i], &rows);
        team_total += tw[i];
        team_max = std::max(team_max, tw[i]);
        lds_ok[i] = batch_lds_bytes(s.dim, s.n_lo, s.n_hi) <= kLdsCap;
    }
    const int n_cu = items[0].ham->basis->ctx->n_cu > 0 ? items[0].ham->basis->ctx->n_cu : 256;
    const bool small = team_max > 1 && team_total <= n_cu;
    std::vector<int> order;   // LDS-kernel requests, then team requests by launch group
    size_t lds_max = 0;
    for (int i = 0; i < n; ++i)
        if (lds_ok[i] && !small) {
            order.push_back(i);
            const Species &s = items[i].ham->basis->sp[0];
            lds_max = std::max(lds_max, batch_lds_bytes(s.dim, s.n_lo, s.n_hi));
        }
    const int n_lds = (int)order.size();
    std::vector<int> grp_first, grp_w;   // team launch groups: first position, workgroups
    for (int i = 0; i < n; ++i) {
        if (lds_ok[i] && !small) continue;
        if (grp_first.empty() || grp_w.back() + tw[i] > n_cu) {
            grp_first.push_back((int)order.size());
            grp_w.push_back(0);
        }
        tbase[i] = grp_w.back();
        grp_w.back() += tw[i];
        order.push_back(i);
    }
    const int n_grp = (int)grp_first.size();
    // one allocation: vectors, alpha/beta, partial sums, then (zeroed
    // together) one arrival ticket per team launch, the team barrier
    // counters and the flags; tickets and counters one per 256-byte line so
    // that polling teams do not share a line
    DevMem work, desc;
    constexpr size_t kLine = 64;   // unsigned per 256-byte line
    const size_t dbytes = (sizeof(double) * (nq + nab + npart) + 255) / 256 * 256;
    const size_t ibytes = sizeof(unsigned) * kLine * ((size_t)n_grp + (size_t)n) + sizeof(int) * 2 * (size_t)n;
    HPHI_TRY(work.alloc(dbytes + ibytes));
    double *qbase = work.as<double>();
    double *abbase = qbase + nq;
    double *partbase = abbase + nab;
    unsigned *tickets = reinterpret_cast<unsigned *>(static_cast<unsigned char *>(work.p) + dbytes);
    unsigned *bar0 = tickets + kLine * (size_t)n_grp;
    int *flags = reinterpret_cast<int *>(bar0 + kLine * (size_t)n);
    HPHI_HIP(hipMemsetAsync(tickets, 0, ibytes, st));
    std::vector<unsigned char> hd(batch_item_size() * (size_t)n);
    for (int p = 0; p < n; ++p) {
        const int i = order[p];
        HPHI_TRY(fill_batch_item(items[i].ham, items[i].max_iter, items[i].seed, qbase + q_off[i],
                                 abbase + ab_off[i], abbase + ab_off[i] + items[i].max_iter, flags + 2 * i,
                                 partbase + part_off[i], bar0 + kLine * i, tbase[i],
                                 hd.data() + batch_item_size() * p));
    }
    HPHI_TRY(desc.alloc(hd.size()));
    HPHI_HIP(hipMemcpyAsync(desc.p, hd.data(), hd.size(), hipMemcpyHostToDevice, st));
    unsigned char *dd = static_cast<unsigned char *>(desc.p);
    if (n_lds > 0) HPHI_TRY(launch_lanczos_batch(dd, n_lds, st, lds_max));
    for (int g = 0; g < n_grp; ++g) {
        const int end = g + 1 < n_grp ? grp_first[g + 1] : n;
        HPHI_TRY(launch_lanczos_team(dd + batch_item_size() * grp_first[g], end - grp_first[g], grp_w[g],
                                     tickets + kLine * g, st));
    }
    std::vector<double> hab(nab);
    std::vector<int> hf(2 * (size_t)n);
    HPHI_HIP(hipMemcpyAsync(hab.data(), abbase, sizeof(double) * nab, hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipMemcpyAsync(hf.data(), flags, sizeof(int) * 2 * n, hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i)
        if (hf[2 * i + 1] == 3) return fail(HPHI_ERR_DEVICE, "item %d: team barrier timed out", i);
    for (int i = 0; i < n; ++i) {
        const double *al = hab.data() + ab_off[i];
        const double *be = al + items[i].max_iter;
        const int k = hf[2 * i];
        items[i].iterations = k;
        items[i].breakdown = hf[2 * i + 1];
        if (items[i].alpha_out) std::memcpy(items[i].alpha_out, al, sizeof(double) * k);
        if (items[i].beta_out) std::memcpy(items[i].beta_out, be, sizeof(double) * k);
        double e = NAN;
        if (k > 0) HPHI_TRY(tridiag_lowest(al, be, k, 1, &e, nullptr));
        items[i].energy = e;
    }
    return HPHI_OK;
}

int hphi_szq(hphi_ham *h, const double *phase, const void *psi_dev, void *b_dev, void *stream)
{
    if (!h || !phase || !psi_dev || !b_dev) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (h->basis->n_sites > 64) return fail(HPHI_ERR_INVALID_ARG, "too many sites");
    DeviceGuard g(h->basis->ctx->device);
    hipStream_t st = (hipStream_t)stream;
    HPHI_USE_HAM(h, st);
    DevMem ph;
    HPHI_TRY(upload(ph, phase, sizeof(double) * 2 * h->basis->n_sites));
    HPHI_TRY(launch_szq(h, ph.as<double>(), psi_dev, b_dev, st));
    HPHI_HIP(hipStreamSynchronize(st));
    return HPHI_OK;
}

// Shifted COCG needs b^T b != 0; a complex excitation such as S^z(q) psi
// with q != 0, pi has b^T b = 0 by momentum conservation (the bilinear form
// pairs momentum q with -q), so the seed system breaks down at once. With H
// real symmetric, (z - H)^-1 is complex symmetric and
//   D(z) = b^H (z - H)^-1 b = D_Re(z) + D_Im(z)
// (the cross terms a^T (z - H)^-1 c and c^T (z - H)^-1 a cancel), where
// D_Re, D_Im come from the real-valued right-hand sides Re b and Im b, for
// which r^T r = |r|^2 > 0. Each nonzero part runs its own Krylov sequence.
int hphi_sqw(hphi_ham *h, const hphi_sqw_opts *o, const void *b_dev, const double *z_re, const double *z_im,
             int n_shift, double *D_out, double *resid_out, hphi_sqw_info *info)
{
    if (!h || !o || !b_dev || !z_re || !z_im || !D_out) return fail(HPHI_ERR_INVALID_ARG, "null argument");
    if (n_shift < 1 || n_shift > 4096) return fail(HPHI_ERR_INVALID_ARG, "n_shift %d outside [1, 4096]", n_shift);
    if (o->max_iter < 1) return fail(HPHI_ERR_INVALID_ARG, "max_iter < 1");
    if (o->seed_shift >= n_shift) return fail(HPHI_ERR_INVALID_ARG, "seed_shift out of range");
    if (h->kind == 1 && h->hub.cplx)
        return fail(HPHI_ERR_UNSUPPORTED, "complex transfers: z - H is not complex symmetric (COCG)");
    DeviceGuard g(h->basis->ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)o->stream;
    HPHI_USE_HAM(h, st);
    const int64_t dim = h->basis->dim;
    const int seed = o->seed_shift >= 0 ? o->seed_shift : n_shift / 2;
    DevMem bp, r, p, hp, cgm, shm;
    HPHI_TRY(bp.alloc(sizeof(double) * 2 * (size_t)dim));
    HPHI_TRY(r.alloc(sizeof(double) * 2 * (size_t)dim));
    HPHI_TRY(p.alloc(sizeof(double) * 2 * (size_t)dim));
    HPHI_TRY(hp.alloc(sizeof(double) * 2 * (size_t)dim));
    CgDev c0{};
    c0.zs = {z_re[seed], z_im[seed]};
    HPHI_TRY(upload(cgm, &c0, sizeof(CgDev)));
    std::vector<ShiftDev> s0(n_shift);
    for (int j = 0; j < n_shift; ++j) {
        s0[j] = ShiftDev{};
        s0[j].sigma = {z_re[j] - z_re[seed], z_im[j] - z_im[seed]};
    }
    HPHI_TRY(upload(shm, s0.data(), sizeof(ShiftDev) * n_shift));
    Reduce red = reduce_at(h, h->red_result.as<double>());
    CgDev hc{};
    // starts the sequence for part `part` of b (r = p = part, shift state
    // reset) and returns |part|^2
    auto start = [&](int part, double *bn2) -> int {
        HPHI_TRY(launch_cplx_part(b_dev, bp.p, dim, part, st));
        HPHI_TRY(launch_cocg_init(bp.p, r.p, p.p, dim, cgm.p, shm.p, n_shift, o->tol, red, st));
        HPHI_HIP(hipMemcpyAsync(&hc, cgm.p, sizeof(CgDev), hipMemcpyDeviceToHost, st));
        HPHI_HIP(hipStreamSynchronize(st));
        *bn2 = hc.bnorm2;
        return HPHI_OK;
    };
    double bn2[2];
    HPHI_TRY(start(1, &bn2[1]));
    HPHI_TRY(start(0, &bn2[0]));           // the real part's sequence is ready
    const double bnorm = std::sqrt(bn2[0] + bn2[1]);
    const double bsum = std::sqrt(bn2[0]) + std::sqrt(bn2[1]);
    // per-part relative tolerance such that |r_Re| + |r_Im| < tol |b|
    const double tol_part = bsum > 0.0 ? o->tol * bnorm / bsum : o->tol;
    std::vector<double> D(2 * n_shift, 0.0), res(n_shift, 0.0);
    std::vector<ShiftDev> s1(n_shift);
    int it_total = 0, converged = 1;
    const int check = 8;
    for (int part = 0; part < 2; ++part) {
        if (bn2[part] == 0.0) continue;     // D_part = 0, nothing to iterate
        // a part below tol |b| (e.g. the rounding of sin(q x) at q = pi) is
        // left out: x_part = 0 leaves the residual |b_part| < tol |b|,
        // which is counted, and changes D by O(|b_part|^2)
        if (std::sqrt(bn2[part]) <= o->tol * bnorm) {
            for (int j = 0; j < n_shift; ++j) res[j] += std::sqrt(bn2[part]) / bnorm;
            continue;
        }
        if (part == 1) {
            double tmp;
            HPHI_TRY(start(1, &tmp));
        }
        int it = 0, conv = 0;
        // spin models on a stored basis: the product's fixed-order dots form
        // mu = p^T (z_s p - H p) and alpha (one vector pass fewer)
        const bool fold_mu = h->kind == 0 && spin_stored_path(h);
        while (it < o->max_iter) {
            MultArgs a{};
            a.dtype = HPHI_C128;
            a.nvec = 1;
            a.v = p.p;
            a.w = hp.p;
            a.red = red;
            a.stream = st;
            if (fold_mu) {
                a.dots = 1;
                a.cocg = cgm.p;
            }
            HPHI_TRY(launch_mult(h, a));
            HPHI_TRY(launch_cocg_iter(r.p, p.p, hp.p, bp.p, dim, cgm.p, shm.p, n_shift, tol_part, red, st, fold_mu));
            ++it;
            if (it % check == 0 || it == o->max_iter) {
                HPHI_HIP(hipMemcpyAsync(&hc, cgm.p, sizeof(CgDev), hipMemcpyDeviceToHost, st));
                HPHI_HIP(hipStreamSynchronize(st));
                if (hc.max_res < tol_part) {
                    conv = 1;
                    break;
                }
                if (hc.breakdown) break;
            }
        }
        HPHI_HIP(hipMemcpyAsync(s1.data(), shm.p, sizeof(ShiftDev) * n_shift, hipMemcpyDeviceToHost, st));
        HPHI_HIP(hipStreamSynchronize(st));
        const double w = std::sqrt(bn2[part]) / bnorm;
        for (int j = 0; j < n_shift; ++j) {
            D[2 * j] += s1[j].X.re;
            D[2 * j + 1] += s1[j].X.im;
            res[j] += s1[j].res * w;        // |r_part| / |b|
        }
        it_total += it;
        converged &= conv;
    }
    double mx = 0.0;
    for (int j = 0; j < n_shift; ++j) {
        D_out[2 * j] = D[2 * j];
        D_out[2 * j + 1] = D[2 * j + 1];
        if (resid_out) resid_out[j] = res[j];
        mx = std::max(mx, res[j]);
    }
    if (info) {
        info->iterations = it_total;
        info->converged = converged;
        info->max_residual = mx;
        info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return HPHI_OK;
}

int hphi_sqw_batch(hphi_ham *const *hams, int n, const hphi_sqw_opts *o, const void *const *b_devs,
                   const double *z_re, const double *z_im, int n_shift, double *D_out, double *resid_out,
                   hphi_sqw_info *info)
{
    if (!hams || n < 1 || !o || !b_devs || !z_re || !z_im || !D_out)
        return fail(HPHI_ERR_INVALID_ARG, "null argument or empty batch");
    if (n_shift < 1 || n_shift > 1024) return fail(HPHI_ERR_INVALID_ARG, "n_shift %d outside [1, 1024]", n_shift);
    if (o->max_iter < 1) return fail(HPHI_ERR_INVALID_ARG, "max_iter < 1");
    if (o->seed_shift >= n_shift) return fail(HPHI_ERR_INVALID_ARG, "seed_shift out of range");
    for (int i = 0; i < n; ++i) {
        if (!hams[i] || !b_devs[i]) return fail(HPHI_ERR_INVALID_ARG, "request %d: null Hamiltonian or b", i);
        if (hams[i]->basis->ctx != hams[0]->basis->ctx)
            return fail(HPHI_ERR_INVALID_ARG, "requests on different contexts");
        if (hams[i]->kind == 1 && hams[i]->hub.cplx)
            return fail(HPHI_ERR_UNSUPPORTED, "request %d: complex transfers (COCG needs a complex-symmetric z - H)", i);
    }
    DeviceGuard g(hams[0]->basis->ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t st = (hipStream_t)o->stream;
    const int seed = o->seed_shift >= 0 ? o->seed_shift : n_shift / 2;
    const int ni = 2 * n;   // item 2 i + part
    // one device allocation: the items' complex vectors, chunk partials,
    // outputs, then the shift records
    std::vector<size_t> vec_off(ni), ch_off(ni);
    size_t nd = 0;
    for (int k = 0; k < ni; ++k) {
        const int64_t dim = hams[k / 2]->basis->dim;
        vec_off[k] = nd;
        nd += 6 * (size_t)dim;
    }
    for (int k = 0; k < ni; ++k) {
        ch_off[k] = nd;
        nd += 5 * (size_t)cocg_chunks(hams[k / 2]->basis->dim);
    }
    const size_t out_off = nd;
    nd += 6 * (size_t)ni;
    nd = (nd + 1) & ~(size_t)1;
    const size_t sh_bytes = sizeof(ShiftDev) * (size_t)n_shift * ni;
    DevMem mem, items;
    HPHI_TRY(mem.alloc(sizeof(double) * nd + sh_bytes));
    double *base = mem.as<double>();
    ShiftDev *sh_dev = reinterpret_cast<ShiftDev *>(base + nd);
    std::vector<ShiftDev> sh((size_t)n_shift * ni);
    std::vector<unsigned char> it((size_t)ni * cocg_item_size());
    for (int k = 0; k < ni; ++k) {
        const int i = k / 2;
        const double *zr = z_re + (size_t)i * n_shift, *zi = z_im + (size_t)i * n_shift;
        for (int j = 0; j < n_shift; ++j) {
            ShiftDev &x = sh[(size_t)k * n_shift + j];
            x = ShiftDev{};
            x.sigma = {zr[j] - zr[seed], zi[j] - zi[seed]};
        }
        const int64_t dim = hams[i]->basis->dim;
        double *v = base + vec_off[k];
        HPHI_TRY(fill_cocg_item(hams[i], b_devs[i], k & 1, v, v + 2 * dim, v + 4 * dim, base + ch_off[k],
                                sh_dev + (size_t)k * n_shift, n_shift, zr[seed], zi[seed], o->tol, o->max_iter,
                                base + out_off + 6 * (size_t)k, it.data() + (size_t)k * cocg_item_size()));
    }
    HPHI_HIP(hipMemcpyAsync(sh_dev, sh.data(), sh_bytes, hipMemcpyHostToDevice, st));
    HPHI_TRY(items.alloc(it.size()));
    HPHI_HIP(hipMemcpyAsync(items.p, it.data(), it.size(), hipMemcpyHostToDevice, st));
    HPHI_TRY(launch_cocg_batch(items.p, ni, st));
    std::vector<double> outs(6 * (size_t)ni);
    HPHI_HIP(hipMemcpyAsync(sh.data(), sh_dev, sh_bytes, hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipMemcpyAsync(outs.data(), base + out_off, sizeof(double) * outs.size(), hipMemcpyDeviceToHost, st));
    HPHI_HIP(hipStreamSynchronize(st));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (int i = 0; i < n; ++i) {
        double *D = D_out + (size_t)i * 2 * n_shift;
        std::vector<double> res(n_shift, 0.0);
        for (int j = 0; j < 2 * n_shift; ++j) D[j] = 0.0;
        int iters = 0, conv = 1;
        for (int part = 0; part < 2; ++part) {
            const int k = 2 * i + part;
            const double *ok = outs.data() + 6 * (size_t)k;
            const double bn2 = ok[3], bnorm = std::sqrt(ok[4]);
            if (bn2 == 0.0 || bnorm == 0.0) continue;
            const double w = std::sqrt(bn2) / bnorm;
            if (ok[5] != 0.0) {   // part below tol |b|: no sequence, its norm joins the residual
                for (int j = 0; j < n_shift; ++j) res[j] += w;
                continue;
            }
            for (int j = 0; j < n_shift; ++j) {
                const ShiftDev &x = sh[(size_t)k * n_shift + j];
                D[2 * j] += x.X.re;
                D[2 * j + 1] += x.X.im;
                res[j] += x.res * w;
            }
            iters += (int)ok[0];
            conv &= ok[1] != 0.0 ? 1 : 0;
        }
        double mx = 0.0;
        for (int j = 0; j < n_shift; ++j) {
            if (resid_out) resid_out[(size_t)i * n_shift + j] = res[j];
            mx = std::max(mx, res[j]);
        }
        if (info) {
            info[i].iterations = iters;
            info[i].converged = conv;
            info[i].max_residual = mx;
            info[i].seconds = secs;
        }
    }
    return HPHI_OK;
}

} // extern "C"

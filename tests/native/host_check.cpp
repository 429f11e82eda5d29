// Host-only checks of the library's C++ pieces, built with g++ and the
// address and undefined-behaviour sanitizers (no GPU needed):
//   tables   the split two-level rank tables against enumeration
//   tridiag  Sturm bisection + inverse iteration on a matrix from stdin
//   guard    the one-user guard of a Hamiltonian's scratch memory
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../paper_2307_13222_amd/csrc/internal.h"

namespace hphi {
// build_species() materializes through a device kernel; only the host
// tables are exercised here.
int launch_materialize(Species &, hipStream_t) { return fail(HPHI_ERR_UNSUPPORTED, "no device"); }
}

using namespace hphi;

static int check_tables()
{
    long checked = 0;
    for (int n = 1; n <= 16; ++n) {
        for (int k = 0; k <= n; ++k) {
            for (int n_lo = 1; n_lo <= n; ++n_lo) {
                Species s;
                if (build_species_tables(s, n, k, n_lo) != HPHI_OK) {
                    std::printf("FAIL build n=%d k=%d n_lo=%d: %s\n", n, k, n_lo, last_error());
                    return 1;
                }
                int64_t r = 0;
                for (uint64_t x = 0; x < (uint64_t(1) << n); ++x) {
                    if (__builtin_popcountll(x) != k) {
                        if (s.rank_of(x) != -1) {
                            std::printf("FAIL outside n=%d k=%d x=%llu\n", n, k, (unsigned long long)x);
                            return 1;
                        }
                        continue;
                    }
                    if (s.rank_of(x) != r || s.state_at(r) != x) {
                        std::printf("FAIL n=%d k=%d n_lo=%d x=%llu r=%lld\n", n, k, n_lo,
                                    (unsigned long long)x, (long long)r);
                        return 1;
                    }
                    ++r;
                    ++checked;
                }
                if (r != s.dim) {
                    std::printf("FAIL dim n=%d k=%d\n", n, k);
                    return 1;
                }
            }
        }
    }
    // rejected inputs
    Species s;
    if (build_species_tables(s, 0, 0, 0) != HPHI_ERR_INVALID_ARG || build_species_tables(s, 8, 9, 0) != HPHI_ERR_INVALID_ARG ||
        build_species_tables(s, 64, 32, 0) != HPHI_ERR_DIM_OVERFLOW) {
        std::printf("FAIL error codes\n");
        return 1;
    }
    std::printf("tables ok %ld\n", checked);
    return 0;
}

static int run_tridiag()
{
    int n = 0, k = 0;
    if (std::scanf("%d %d", &n, &k) != 2 || n < 1 || k < 1 || k > n) return 2;
    std::vector<double> a(n), b(n);
    for (int i = 0; i < n; ++i)
        if (std::scanf("%lf", &a[i]) != 1) return 2;
    for (int i = 0; i < n; ++i)
        if (std::scanf("%lf", &b[i]) != 1) return 2;
    std::vector<double> ev(k), vec(n);
    if (tridiag_lowest(a.data(), b.data(), n, k, ev.data(), vec.data()) != HPHI_OK) return 3;
    for (double e : ev) std::printf("%.17g\n", e);
    for (double v : vec) std::printf("%.17g\n", v);
    return 0;
}

// Fake device side: events are counters of unfinished work per stream.
struct FakeOps {
    int pending_work = 0;       // work of the last recorded call still running
    bool capture = false;
    bool pending(void *) { return pending_work > 0; }
    void record(void *, void *) {}
    bool capturing(void *) { return capture; }
};

#define EXPECT(c)                                            \
    do {                                                     \
        if (!(c)) {                                          \
            std::printf("FAIL guard line %d: %s\n", __LINE__, #c); \
            return 1;                                        \
        }                                                    \
    } while (0)

static int check_guard()
{
    UseState st;
    int ev_obj = 0;
    st.event = &ev_obj;
    FakeOps ops;
    void *s1 = (void *)0x10, *s2 = (void *)0x20;
    {
        UseScope<FakeOps> a(st, ops, s1);
        EXPECT(a.verdict() == USE_OK);
        // a second call while the first is inside: another host thread
        UseScope<FakeOps> b(st, ops, s1);
        EXPECT(b.verdict() == USE_OTHER_THREAD);
    }
    EXPECT(st.busy.load() == 0 && st.recorded && st.last_stream == s1);
    ops.pending_work = 1;   // the first call's kernels still run on s1
    {
        UseScope<FakeOps> c(st, ops, s1);   // same stream: queues in order
        EXPECT(c.verdict() == USE_OK);
    }
    {
        UseScope<FakeOps> d(st, ops, s2);   // another stream while s1 runs
        EXPECT(d.verdict() == USE_OTHER_STREAM);
    }
    EXPECT(st.busy.load() == 0 && st.last_stream == s1);
    ops.capture = true;     // graph capture: the caller orders replays
    {
        UseScope<FakeOps> e(st, ops, s2);
        EXPECT(e.verdict() == USE_OK);
    }
    EXPECT(st.last_stream == s1);   // nothing recorded while capturing
    ops.capture = false;
    ops.pending_work = 0;   // s1 drained (synchronized)
    {
        UseScope<FakeOps> f(st, ops, s2);
        EXPECT(f.verdict() == USE_OK);
    }
    EXPECT(st.last_stream == s2);
    // without an event there is no stream check, only the thread check
    UseState nost;
    ops.pending_work = 1;
    {
        UseScope<FakeOps> g(nost, ops, s1);
        EXPECT(g.verdict() == USE_OK);
    }
    {
        UseScope<FakeOps> h(nost, ops, s2);
        EXPECT(h.verdict() == USE_OK);
    }
    std::printf("guard ok\n");
    return 0;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    if (!std::strcmp(argv[1], "tables")) return check_tables();
    if (!std::strcmp(argv[1], "tridiag")) return run_tridiag();
    if (!std::strcmp(argv[1], "guard")) return check_guard();
    return 2;
}

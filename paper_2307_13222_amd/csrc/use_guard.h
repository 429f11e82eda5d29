// One-user guard of a Hamiltonian's scratch memory (reduction partials,
// completion counters, work queues), which every call on that Hamiltonian
// uses. A call may start when no other host thread is inside a call on it
// and, if the previous call ran on another stream, that call's work has
// finished. The device side is abstracted by Ops so the logic builds and is
// tested without a GPU:
//   bool pending(void *event)           recorded work not finished yet
//   void record(void *event, void *st)  mark the end of this call's work
//   bool capturing(void *st)            stream under graph capture
#pragma once

#include <atomic>

namespace hphi {

struct UseState {
    std::atomic<int> busy{0};
    void *event = nullptr;       // null: no stream check (event unavailable)
    void *last_stream = nullptr;
    bool recorded = false;
};

enum UseVerdict { USE_OK = 0, USE_OTHER_THREAD = 1, USE_OTHER_STREAM = 2 };

template <class Ops>
class UseScope {
public:
    UseScope(UseState &s, Ops &ops, void *stream) : s_(s), ops_(ops), stream_(stream)
    {
        int expected = 0;
        if (!s_.busy.compare_exchange_strong(expected, 1, std::memory_order_acquire)) {
            verdict_ = USE_OTHER_THREAD;
            return;
        }
        held_ = true;
        capturing_ = ops_.capturing(stream_);
        if (!capturing_ && s_.event && s_.recorded && s_.last_stream != stream_ && ops_.pending(s_.event)) {
            verdict_ = USE_OTHER_STREAM;
            release();
        }
    }
    ~UseScope()
    {
        if (!held_) return;
        if (!capturing_ && s_.event) {
            ops_.record(s_.event, stream_);
            s_.last_stream = stream_;
            s_.recorded = true;
        }
        release();
    }
    UseScope(const UseScope &) = delete;
    UseScope &operator=(const UseScope &) = delete;
    UseVerdict verdict() const { return verdict_; }

private:
    void release()
    {
        held_ = false;
        s_.busy.store(0, std::memory_order_release);
    }
    UseState &s_;
    Ops &ops_;
    void *stream_;
    UseVerdict verdict_ = USE_OK;
    bool held_ = false;
    bool capturing_ = false;
};

} // namespace hphi

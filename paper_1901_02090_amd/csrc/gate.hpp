// Process-wide gate between stream captures and other threads' HIP calls.
#pragma once
#include <condition_variable>
#include <mutex>
#include <shared_mutex>

namespace bddc {

// A stream capture must not overlap HIP calls of other threads that allocate,
// free, copy synchronously or synchronise (each has invalidated a capture in
// flight here).  Captures take this gate exclusively; every other path of the
// library that calls HIP holds it shared.  Waiting writers stop new readers,
// so a capture is not starved by a busy server driver.
class HipGate {
  std::mutex m_;
  std::condition_variable cv_;
  int readers_ = 0, waiting_ = 0;
  bool writer_ = false;

 public:
  void lock_shared() {
    std::unique_lock<std::mutex> lk(m_);
    cv_.wait(lk, [&] { return !writer_ && waiting_ == 0; });
    ++readers_;
  }
  void unlock_shared() {
    std::lock_guard<std::mutex> lk(m_);
    if (--readers_ == 0) cv_.notify_all();
  }
  void lock() {
    std::unique_lock<std::mutex> lk(m_);
    ++waiting_;
    cv_.wait(lk, [&] { return !writer_ && readers_ == 0; });
    --waiting_;
    writer_ = true;
  }
  void unlock() {
    std::lock_guard<std::mutex> lk(m_);
    writer_ = false;
    cv_.notify_all();
  }
};
inline HipGate g_gate;
using GateShared = std::shared_lock<HipGate>;
using GateExclusive = std::unique_lock<HipGate>;

}  // namespace bddc

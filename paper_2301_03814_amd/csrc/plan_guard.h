// One host thread at a time inside the calls on a plan.
//
// Host code only, no HIP: the flag is a plain int owned by the plan (so that
// the plan object stays copyable) and is taken with an atomic exchange.  A
// call that finds it taken does not wait: it reports the plan as busy.
#pragma once

namespace swkb {

class PlanGuard {
 public:
  explicit PlanGuard(int* flag) : flag_(flag), held_(__atomic_exchange_n(flag, 1, __ATOMIC_ACQUIRE) == 0) {}
  ~PlanGuard() {
    if (held_) __atomic_store_n(flag_, 0, __ATOMIC_RELEASE);
  }
  PlanGuard(const PlanGuard&) = delete;
  PlanGuard& operator=(const PlanGuard&) = delete;
  // false: another thread holds the plan; the caller must not touch it
  bool held() const { return held_; }

 private:
  int* flag_;
  bool held_;
};

}  // namespace swkb

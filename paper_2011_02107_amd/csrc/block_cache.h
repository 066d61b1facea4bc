// Stream-ordered cache of device blocks, shared by host threads that each drive their own stream.
//
// A freed block carries an event recorded on the freeing thread's stream; the next user's stream
// waits on that event before the block is handed out, so reuse is ordered behind every earlier use
// on the freeing stream.  Events of blocks handed out go back to a spare list for later frees.
//
// The runtime calls are a template parameter (Rt), so the same hand-off logic runs on the HIP
// runtime in the library and on a recording stand-in in the host-side test harness.  Rt provides:
//   types Stream, Event, Err; constants ok, oom (Err values);
//   Err malloc(void **p, size_t n); void free(void *p);
//   Err event_create(Event *e); Err record(Event e, Stream s); Err wait(Stream s, Event e).
#pragma once

#include <algorithm>
#include <cstddef>
#include <map>
#include <mutex>
#include <vector>

namespace dacp {

template <class Rt>
class BlockCacheT {
 public:
  using Stream = typename Rt::Stream;
  using Event = typename Rt::Event;
  using Err = typename Rt::Err;

  explicit BlockCacheT(size_t limit_bytes) : limit_(limit_bytes) {}

  // Size class: n rounded up to a multiple of a quarter of its leading power of two (256 B at least).
  static size_t size_class(size_t n) {
    size_t top = 256;
    while (top * 2 <= n) top *= 2;
    const size_t step = std::max<size_t>(256, top / 4);
    return (n + step - 1) / step * step;
  }

  // A block of at least n bytes usable on stream s (cls gets its size class).
  Err alloc(Rt &rt, size_t n, Stream s, void **p, size_t *cls) {
    const size_t c = size_class(n);
    *cls = c;
    {
      std::unique_lock<std::mutex> lk(mu_);
      auto it = blocks_.find(c);
      if (it != blocks_.end()) {
        const Cached b = it->second;
        blocks_.erase(it);
        cached_ -= c;
        // The wait is queued before the event goes back to the spare list, with the lock held:
        // a free on another thread can take the event from the list and record it on its own
        // stream only after this wait has captured the freeing stream's point.  Queued after the
        // unlock, the wait could see that later record and hand the block out while its previous
        // stream still uses it, and one event would be recorded and waited on by two threads at
        // once.
        const Err e = rt.wait(s, b.ready);
        spare_.push_back(b.ready);
        lk.unlock();
        if (e != Rt::ok) {
          rt.free(b.p);  // the runtime's free waits for the device, so the block's last use is over
          return e;
        }
        *p = b.p;
        return Rt::ok;
      }
    }
    Err e = rt.malloc(p, c);
    if (e == Rt::oom) {
      // hand every cached block back to the runtime, then try once more
      bool had = false;
      {
        std::lock_guard<std::mutex> lk(mu_);
        had = !blocks_.empty();
      }
      if (had) {
        trim(rt);
        e = rt.malloc(p, c);
      }
    }
    return e;
  }

  // Return block p (size class cls) after its last use on stream s.
  void release(Rt &rt, void *p, size_t cls, Stream s) {
    Event ev{};
    bool have_ev = false, keep;
    {
      std::lock_guard<std::mutex> lk(mu_);
      keep = cached_ + cls <= limit_;
      if (keep) {
        cached_ += cls;  // reserved until the block is filed below or released
        if (!spare_.empty()) {
          ev = spare_.back();
          spare_.pop_back();
          have_ev = true;
        }
      }
    }
    if (keep && !have_ev) have_ev = rt.event_create(&ev) == Rt::ok;
    if (keep && have_ev && rt.record(ev, s) == Rt::ok) {
      std::lock_guard<std::mutex> lk(mu_);
      blocks_.insert({cls, Cached{p, ev}});
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      if (keep) cached_ -= cls;
      if (have_ev) spare_.push_back(ev);
    }
    rt.free(p);
  }

  // Hand every cached block back to the runtime (whose free waits for the device).
  void trim(Rt &rt) {
    std::vector<void *> held;
    {
      std::lock_guard<std::mutex> lk(mu_);
      for (const auto &kv : blocks_) {
        held.push_back(kv.second.p);
        spare_.push_back(kv.second.ready);
        cached_ -= kv.first;  // bytes reserved by a release still in progress stay counted
      }
      blocks_.clear();
    }
    for (void *q : held) rt.free(q);
  }

  size_t cached_bytes() {
    std::lock_guard<std::mutex> lk(mu_);
    return cached_;
  }

 private:
  struct Cached {
    void *p;
    Event ready;  // recorded on the freeing stream
  };
  std::mutex mu_;
  std::multimap<size_t, Cached> blocks_;  // by size class
  std::vector<Event> spare_;              // events not attached to a block
  size_t cached_ = 0;
  size_t limit_;
};

}  // namespace dacp

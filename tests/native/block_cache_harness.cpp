// Host-side harness of the library's block cache (paper_2011_02107_amd/csrc/block_cache.h) on a
// recording stand-in for the runtime: no device.  Many threads, each with its own "stream",
// allocate, use and free blocks of a few size classes.  The stand-in checks the hand-off rule the
// cache promises: when a block is handed to a new stream, that stream's wait captures exactly the
// event state recorded when the block was last freed (so reuse is ordered behind every earlier use),
// and no event is recorded while a wait on it is being queued.  Build with -fsanitize=thread (data
// races) or -fsanitize=address,undefined.  Exit status 0 = every check held.
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "block_cache.h"

namespace {

struct MockEvent {
  std::mutex mu;
  unsigned long long token = 0;  // state captured by the latest record
  std::atomic<int> waiting{0};   // waits being queued right now
};

std::atomic<int> g_failures{0};
std::atomic<unsigned long long> g_next_token{1};
std::mutex g_side_mu;
std::unordered_map<void *, unsigned long long> g_freed_token;  // block -> token of its last free
thread_local void *t_releasing = nullptr;                      // block being released by this thread
thread_local unsigned long long t_wait_token = 0;              // token the latest wait captured
std::vector<MockEvent *> g_events;
std::mutex g_events_mu;

void fail(const char *what) {
  if (g_failures.fetch_add(1) < 10) std::fprintf(stderr, "FAIL: %s\n", what);
}

struct MockRt {
  using Stream = int;
  using Event = MockEvent *;
  using Err = int;
  static constexpr int ok = 0;
  static constexpr int oom = 2;

  int malloc(void **p, size_t n) {
    *p = std::malloc(n);
    return *p ? ok : oom;
  }
  void free(void *p) { std::free(p); }
  int event_create(MockEvent **e) {
    *e = new MockEvent;
    std::lock_guard<std::mutex> lk(g_events_mu);
    g_events.push_back(*e);
    return ok;
  }
  int record(MockEvent *e, int) {
    if (e->waiting.load() != 0) fail("an event was recorded while a wait on it was being queued");
    unsigned long long t;
    {
      std::lock_guard<std::mutex> lk(e->mu);
      t = e->token = g_next_token.fetch_add(1);
    }
    std::lock_guard<std::mutex> lk(g_side_mu);
    g_freed_token[t_releasing] = t;
    return ok;
  }
  int wait(int, MockEvent *e) {
    e->waiting.fetch_add(1);
    std::this_thread::yield();  // widen the window in which a misplaced record would land
    {
      std::lock_guard<std::mutex> lk(e->mu);
      t_wait_token = e->token;
    }
    std::this_thread::yield();
    e->waiting.fetch_sub(1);
    return ok;
  }
};

}  // namespace

int main() {
  dacp::BlockCacheT<MockRt> cache(size_t(1) << 20);
  const int threads = 16, iters = 4000;
  std::atomic<long> reused{0};
  std::vector<std::thread> ts;
  for (int t = 0; t < threads; ++t) {
    ts.emplace_back([&, t] {
      MockRt rt;
      unsigned s = 12345u + 7919u * static_cast<unsigned>(t);
      for (int i = 0; i < iters; ++i) {
        s = s * 1103515245u + 12345u;
        const size_t n = size_t(256) << ((s >> 16) % 4);
        void *p = nullptr;
        size_t cls = 0;
        t_wait_token = 0;
        if (cache.alloc(rt, n, t, &p, &cls) != MockRt::ok || !p) {
          fail("alloc failed");
          continue;
        }
        if (cls < n) fail("size class below the request");
        unsigned long long expect = 0;
        {
          std::lock_guard<std::mutex> lk(g_side_mu);
          auto it = g_freed_token.find(p);
          if (it != g_freed_token.end()) {
            expect = it->second;
            g_freed_token.erase(it);
          }
        }
        if (expect) {
          ++reused;
          // this stream's wait must have captured the record made when the block was last freed
          if (t_wait_token != expect) fail("a reused block was ordered behind the wrong point");
        }
        static_cast<unsigned char *>(p)[cls - 1] = static_cast<unsigned char>(t);  // use the block
        t_releasing = p;
        cache.release(rt, p, cls, t);
        t_releasing = nullptr;
      }
    });
  }
  for (auto &th : ts) th.join();
  {
    MockRt rt;
    cache.trim(rt);
    if (cache.cached_bytes() != 0) fail("trim left cached bytes");
  }
  std::printf("block cache harness: %ld reused blocks, %d failures\n", reused.load(), g_failures.load());
  for (MockEvent *e : g_events) delete e;
  if (reused.load() < 1000) {
    std::fprintf(stderr, "FAIL: too few reused blocks to exercise the hand-off\n");
    return 1;
  }
  return g_failures.load() == 0 ? 0 : 1;
}

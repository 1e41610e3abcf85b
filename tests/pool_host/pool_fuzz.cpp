// Random admission / tick / poll / progress sequences through the serving
// pool on the host-only runtime model (mock_runtime.cpp).  Checks, per seed:
// every admitted job is harvested exactly once, after exactly its iteration
// count, with its own result; the arena's free space always equals its size
// minus the live jobs' blocks; no job's work runs on another job's workspace;
// destroying the pool with jobs in flight is clean.  Memory errors are left
// to the sanitizer.  Usage: pool_fuzz SEED [SEED ...]
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>

#include "../../include/lfsr.h"

extern "C" void mock_progress(size_t n);
extern "C" size_t mock_pending();
extern "C" void mock_fail_memcpy_in(long n);
extern "C" void mock_fail_query_in(long n);

namespace {

[[noreturn]] void fail(unsigned seed, const char* what) {
  std::fprintf(stderr, "seed %u: %s\n", seed, what);
  std::exit(1);
}

struct Job {
  int n_iter;
  size_t bytes;
  float *y, *disp, *out;
};

size_t round256(size_t v) { return (v + 255) & ~(size_t)255; }

void run(unsigned seed) {
  std::mt19937 rng(seed);
  const size_t arena_bytes = round256(48 * 1024 + rng() % (256 * 1024));
  void* arena = std::aligned_alloc(256, arena_bytes);
  const int max_slots = 1 + (int)(rng() % 8);
  lfsr_pool* p = nullptr;
  if (lfsr_pool_create(arena, arena_bytes, max_slots, &p) != LFSR_OK) fail(seed, "pool_create");
  const int total = 120;
  const int abandon_at = (seed % 4 == 3) ? (int)(rng() % total) : -1;  // destroy with jobs in flight
  // seeds 5k+4: one runtime call fails part-way (a result copy in tick, or an
  // event query in poll); the pool reports LFSR_EDEVICE and is then destroyed
  const bool inject = seed % 5 == 4;
  if (inject) {
    if (rng() % 2) mock_fail_memcpy_in((long)(rng() % 40));
    else mock_fail_query_in((long)(rng() % 400));
  }
  bool failed = false;
  std::map<int64_t, Job> live;
  size_t live_bytes = 0;
  int submitted = 0, harvested = 0;
  for (long step = 0; harvested < total; ++step) {
    if (step > 2000000) fail(seed, "no progress");
    if (abandon_at >= 0 && harvested >= abandon_at && !live.empty()) break;
    const unsigned a = rng() % 10;
    if (a < 3 && submitted < total) {
      lfsr_params prm{};
      prm.lr_h = 1 + (int)(rng() % 24);
      prm.lr_w = 1 + (int)(rng() % 24);
      prm.admm_iters = 1 + (int)(rng() % 7);
      Job j{prm.admm_iters, round256(lfsr_workspace_bytes(&prm)), new float[4](), new float[4](), new float[4]()};
      j.out[0] = -1.f;
      int64_t id = 0;
      const lfsr_status st = lfsr_pool_submit(p, &prm, j.y, j.disp, nullptr, nullptr, j.out, nullptr, &id);
      if (st == LFSR_OK) {
        if (live.count(id)) fail(seed, "job id reused");
        live[id] = j;
        live_bytes += j.bytes;
        ++submitted;
      } else {
        if (st != LFSR_EBUSY) fail(seed, "submit failed with an unexpected status");
        delete[] j.y;
        delete[] j.disp;
        delete[] j.out;
      }
    } else if (a < 6) {
      int32_t act = -1;
      const lfsr_status st = lfsr_pool_tick(p, nullptr, &act);
      if (st != LFSR_OK) {
        if (!inject || st != LFSR_EDEVICE) fail(seed, "tick");
        failed = true;
        break;
      }
    } else if (a < 8) {
      int64_t ids[8];
      int32_t sts[8], its[8], n = -1;
      const int cap = 1 + (int)(rng() % 8);
      const lfsr_status pst = lfsr_pool_poll(p, ids, sts, its, cap, &n);
      if (pst != LFSR_OK && (!inject || pst != LFSR_EDEVICE)) fail(seed, "poll");
      if (n < 0 || n > cap) fail(seed, "poll count out of range (it is set on errors too)");
      for (int i = 0; i < n; ++i) {
        auto it = live.find(ids[i]);
        if (it == live.end()) fail(seed, "harvested an unknown or already harvested job");
        const Job& j = it->second;
        if (sts[i] != LFSR_OK) fail(seed, "job status not OK");
        if (its[i] != j.n_iter) fail(seed, "iterations reported differ from the job's count");
        if (j.out[0] != (float)j.n_iter) fail(seed, "job output is not its own result after its iterations");
        live_bytes -= j.bytes;
        delete[] j.y;
        delete[] j.disp;
        delete[] j.out;
        live.erase(it);
        ++harvested;
      }
      if (pst != LFSR_OK) {
        failed = true;
        break;
      }
    } else {
      mock_progress(rng() % 48);
    }
    int32_t na = 0, nr = 0;
    size_t fr = 0, big = 0;
    if (lfsr_pool_info(p, &na, &nr, &fr, &big) != LFSR_OK) fail(seed, "info");
    if (fr + live_bytes != arena_bytes) fail(seed, "arena free space does not match the live jobs");
    if (big > fr || (size_t)(na + nr) != live.size()) fail(seed, "pool counts inconsistent");
  }
  mock_fail_memcpy_in(-1);
  mock_fail_query_in(-1);
  (void)failed;
  lfsr_pool_destroy(p);
  mock_progress((size_t)-1);
  if (mock_pending() != 0) fail(seed, "device work left after destroy");
  for (auto& kv : live) {
    delete[] kv.second.y;
    delete[] kv.second.disp;
    delete[] kv.second.out;
  }
  std::free(arena);
}

}  // namespace

int main(int argc, char** argv) {
  for (int i = 1; i < argc; ++i) run((unsigned)std::strtoul(argv[i], nullptr, 10));
  std::printf("pool_fuzz: %d seeds ok\n", argc - 1);
  return 0;
}

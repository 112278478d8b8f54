// Drives the library's host code (the C ABI in api.cpp, the host co-rank,
// the serving runtime in server.cpp) under AddressSanitizer +
// UndefinedBehaviorSanitizer, or under ThreadSanitizer, on a machine with no
// GPU: linked with hip_stub.cpp (the HIP runtime calls, completing at once)
// and launch_stub.cpp (kernel launches that do nothing).  What it checks is
// host logic only: argument checks and their status codes, workspace and
// batch bookkeeping, the tuning table, the host co-rank against a count,
// and the serving runtime's scheduling under several client threads (every
// ticket reported once, the arena empty at the end, shutdown cancelling what
// can no longer run).  Exit status 0 when every check holds.
// Test infrastructure only.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <random>
#include <set>
#include <thread>
#include <vector>

#include "corank_merge.h"

static int g_failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_failures;                                                   \
    }                                                                 \
  } while (0)

// Host buffers standing in for device arrays (the stub launchers never touch
// them; only their addresses and sizes matter to the host code).
struct Buf {
  std::vector<uint64_t> words;
  explicit Buf(size_t bytes) : words(bytes / 8 + 2) {}
  void* p() { return words.data(); }
  size_t bytes() const { return (words.size() - 2) * 8; }
};

static void abi_calls() {
  const uint64_t m = 100000, n = 70001, N = m + n;
  Buf A(m * 8), B(n * 8), Av(m * 8), Bv(n * 8), C(N * 8), Cv(N * 8);
  // merges of every key type, keys only and with 4- and 8-byte payloads,
  // in every boundary mode
  for (int kt = 0; kt < 6; ++kt) {
    const size_t ws_bytes = cm_merge_workspace_size(kt, 1, m, n);
    CHECK(ws_bytes > 0 && ws_bytes % 256 == 0);
    Buf ws(ws_bytes);
    for (int part = -1; part <= 4; ++part) {
      CHECK(cm_set_partition(part) == CM_OK);
      CHECK(cm_stable_merge(kt, A.p(), m, B.p(), n, C.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
      CHECK(cm_stable_merge_pairs(kt, A.p(), (const uint32_t*)Av.p(), m, B.p(), (const uint32_t*)Bv.p(), n, C.p(),
                                  (uint32_t*)Cv.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
      CHECK(cm_stable_merge_pairs64(kt, A.p(), (const uint64_t*)Av.p(), m, B.p(), (const uint64_t*)Bv.p(), n, C.p(),
                                    (uint64_t*)Cv.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
    }
    CHECK(cm_set_partition(-1) == CM_OK);
    // errors: workspace too small, output over an input, null with length
    CHECK(cm_stable_merge(kt, A.p(), m, B.p(), n, C.p(), ws.p(), ws_bytes - 8, nullptr) == CM_ENOSPC);
    CHECK(cm_stable_merge(kt, A.p(), m, B.p(), n, A.p(), ws.p(), ws_bytes, nullptr) == CM_EALIAS);
    CHECK(cm_stable_merge(kt, nullptr, m, B.p(), n, C.p(), ws.p(), ws_bytes, nullptr) == CM_EINVAL);
  }
  CHECK(cm_stable_merge(7, A.p(), m, B.p(), n, C.p(), nullptr, 0, nullptr) == CM_EDTYPE);
  // the allocation-free variant: same checks, the scratch array's limit
  CHECK(cm_stable_merge_pairs_noalloc(0, A.p(), (const uint32_t*)Av.p(), m, B.p(), (const uint32_t*)Bv.p(), n, C.p(),
                                      (uint32_t*)Cv.p(), nullptr) == CM_OK);
  CHECK(cm_stable_merge_pairs_noalloc(0, A.p(), nullptr, m, B.p(), nullptr, n, C.p(), nullptr, nullptr) == CM_OK);
  CHECK(cm_stable_merge_pairs_noalloc(0, A.p(), nullptr, 1ull << 40, B.p(), nullptr, n, C.p(), nullptr, nullptr) ==
        CM_ENOSPC);
  CHECK(cm_stable_merge_pairs_noalloc(0, A.p(), nullptr, m, B.p(), nullptr, n, A.p(), nullptr, nullptr) == CM_EALIAS);
  // grids, block orders, strides and lanes
  const size_t ws_bytes = cm_merge_workspace_size(0, 1, m, n);
  Buf ws(ws_bytes);
  for (int grid : {0, -1, 1, 300}) {
    CHECK(cm_set_grid(grid) == CM_OK);
    for (int order : {0, 1, 32}) {
      CHECK(cm_set_block_order(order) == CM_OK);
      CHECK(cm_stable_merge(0, A.p(), m, B.p(), n, C.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
    }
  }
  CHECK(cm_set_grid(-2) == CM_EINVAL);
  CHECK(cm_set_grid(0) == CM_OK && cm_set_block_order(32) == CM_OK);
  for (int c = -1; c < cm_config_count(); ++c) {
    CHECK(cm_set_config(0, 1, c) == CM_OK);
    CHECK(cm_get_config(0, 1) == c);
    CHECK(cm_stable_merge_pairs(0, A.p(), (const uint32_t*)Av.p(), m, B.p(), (const uint32_t*)Bv.p(), n, C.p(),
                                (uint32_t*)Cv.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
  }
  CHECK(cm_set_config(0, 1, -1) == CM_OK && cm_set_config(0, 1, 99) == CM_ECONFIG);

  // co-rank on the device (stub) and on the host
  std::vector<uint64_t> ranks = {0, 5, N}, js(3);
  CHECK(cm_co_rank(0, ranks.data(), 3, A.p(), m, B.p(), n, js.data(), nullptr) == CM_OK);

  // segmented batch
  const uint64_t S = 1000;
  std::vector<uint64_t> a_off(S + 1), b_off(S + 1);
  for (uint64_t s = 0; s <= S; ++s) {
    a_off[s] = s * m / S;
    b_off[s] = s * n / S;
  }
  const size_t sws = cm_segmented_workspace_size(0, 1, m, n, S);
  Buf sw(sws);
  for (int part : {0, 2}) {
    CHECK(cm_set_partition(part) == CM_OK);
    CHECK(cm_stable_merge_segmented(0, A.p(), (const uint32_t*)Av.p(), a_off.data(), m, B.p(),
                                    (const uint32_t*)Bv.p(), b_off.data(), n, S, C.p(), (uint32_t*)Cv.p(), sw.p(), sws,
                                    nullptr) == CM_OK);
  }
  CHECK(cm_set_partition(-1) == CM_OK);
  CHECK(cm_stable_merge_segmented_each(0, A.p(), (const uint32_t*)Av.p(), a_off.data(), m, B.p(),
                                       (const uint32_t*)Bv.p(), b_off.data(), n, S, C.p(), (uint32_t*)Cv.p(), ws.p(),
                                       ws_bytes, nullptr) == CM_OK);

  // batches: inline descriptors and an uploaded copy, every boundary mode
  for (uint32_t count : {1u, 5u, 16u, 40u}) {
    std::vector<cm_merge_desc> d(count);
    std::vector<Buf> bufs;
    bufs.reserve(3 * count);
    for (uint32_t r = 0; r < count; ++r) {
      const uint64_t mr = (r * 7919) % 5000, nr = (r * 104729) % 3000;
      bufs.emplace_back(mr * 4 + 8);
      bufs.emplace_back(nr * 4 + 8);
      bufs.emplace_back((mr + nr) * 4 + 8);
      d[r] = cm_merge_desc{};
      d[r].A = bufs[3 * r].p();
      d[r].m = mr;
      d[r].B = bufs[3 * r + 1].p();
      d[r].n = nr;
      d[r].C = bufs[3 * r + 2].p();
    }
    uint64_t total = 0;
    CHECK(cm_batch_prepare(0, 0, d.data(), count, &total) == CM_OK);
    const size_t bws = cm_batch_workspace_size(total, count);
    Buf bw(bws);
    std::vector<cm_merge_desc> dev = d;
    for (int part : {0, 1, 2, 4}) {
      CHECK(cm_set_partition(part) == CM_OK);
      CHECK(cm_stable_merge_batch(0, 0, d.data(), dev.data(), count, total, bw.p(), bws, nullptr) == CM_OK);
      const int inline_rc = cm_stable_merge_batch(0, 0, d.data(), nullptr, count, total, bw.p(), bws, nullptr);
      CHECK(inline_rc == (count <= CM_BATCH_INLINE_MAX ? CM_OK : CM_EINVAL));
    }
    CHECK(cm_set_partition(-1) == CM_OK);
  }

  // sort, ablation, records, checks, copies
  const size_t sortws = cm_sort_workspace_size(0, 1, N);
  Buf so(sortws);
  CHECK(cm_stable_sort_pairs(0, A.p(), (const uint32_t*)Av.p(), N / 2, C.p(), (uint32_t*)Cv.p(), so.p(), sortws,
                             nullptr) == CM_OK);
  CHECK(cm_stable_sort(0, C.p(), N / 2, C.p(), so.p(), sortws, nullptr) == CM_OK);  // in place
  uint64_t bounds[2049];
  const size_t aws = cm_partition_ablation_workspace_size(2048);
  Buf ab(aws);
  for (int p : {0, 1})
    CHECK(cm_merge_partition_ablation(0, A.p(), nullptr, m, B.p(), nullptr, n, C.p(), nullptr, 2048, p, bounds, ab.p(),
                                      aws, nullptr) == CM_OK);
  CHECK(cm_origin_codes(m, n, (uint32_t*)Av.p(), (uint32_t*)Bv.p(), nullptr) == CM_OK);
  uint32_t flag = 0;
  CHECK(cm_check_sorted(0, A.p(), m, &flag, nullptr) == CM_OK);
  CHECK(cm_copy(A.p(), C.p(), 4096, nullptr) == CM_OK);
  CHECK(cm_copy_tiles(0, A.p(), (const uint32_t*)Av.p(), 4000, B.p(), (const uint32_t*)Bv.p(), 4000, C.p(),
                      (uint32_t*)Cv.p(), nullptr) == CM_OK);

  // per-call timing
  CHECK(cm_timing_start(8) == CM_OK);
  for (int r = 0; r < 10; ++r)
    CHECK(cm_stable_merge(0, A.p(), m, B.p(), n, C.p(), ws.p(), ws_bytes, nullptr) == CM_OK);
  uint32_t calls = 0;
  double co = 0, me = 0;
  float starts[8], each[8], merges[8];
  CHECK(cm_timing_stop(&calls, &co, &me, starts, each, merges) == CM_OK);
  CHECK(calls == 8);

  // autotuner, tuning table, plans (graph capture fails here: error path)
  int best[3];
  CHECK(cm_autotune_merge(0, A.p(), (const uint32_t*)Av.p(), m, B.p(), (const uint32_t*)Bv.p(), n, C.p(),
                          (uint32_t*)Cv.p(), ws.p(), ws_bytes, 1, nullptr, best) == CM_OK);
  CHECK(cm_autotune_segmented(0, A.p(), (const uint32_t*)Av.p(), a_off.data(), m, B.p(), (const uint32_t*)Bv.p(),
                              b_off.data(), n, S, C.p(), (uint32_t*)Cv.p(), sw.p(), sws, 1, nullptr, best) == CM_OK);
  CHECK(cm_tuning_count() == 2);
  char path[] = "/tmp/cm_sanitize_tuning_XXXXXX";
  const int fd = mkstemp(path);
  CHECK(fd >= 0);
  CHECK(cm_tuning_save(path) == CM_OK);
  CHECK(cm_tuning_clear() == CM_OK && cm_tuning_load(path) == CM_OK && cm_tuning_count() == 2);
  FILE* f = fopen(path, "a");
  fputs("0 0 1 10 99 0 0 1.0\n", f);
  fclose(f);
  CHECK(cm_tuning_load(path) == CM_EINVAL);
  remove(path);
  int choice[3];
  CHECK(cm_tuning_get(2, 0, 1, 1 << 20, choice) == CM_OK);
  CHECK(cm_tuning_clear() == CM_OK);
  cm_plan* plan = nullptr;
  CHECK(cm_plan_create_merge(0, A.p(), nullptr, m, B.p(), nullptr, n, C.p(), nullptr, ws.p(), ws_bytes, &plan) ==
        CM_EHIP);
  CHECK(plan == nullptr);
  CHECK(strlen(cm_status_string(CM_ESTALE)) > 0 && strlen(cm_build_id()) > 0);
}

// cm_co_rank_host against a count of A-origin outputs of the merge, on
// random sorted arrays of a small alphabet (both orders).
static void host_co_rank() {
  std::mt19937_64 rng(7);
  for (int rep = 0; rep < 300; ++rep) {
    const uint64_t m = rng() % 40, n = rng() % 40;
    const bool desc = rep & 1;
    std::vector<uint32_t> A(m), B(n);
    for (auto& x : A) x = (uint32_t)(rng() % 5);
    for (auto& x : B) x = (uint32_t)(rng() % 5);
    std::sort(A.begin(), A.end());
    std::sort(B.begin(), B.end());
    if (desc) {
      std::reverse(A.begin(), A.end());
      std::reverse(B.begin(), B.end());
    }
    for (uint64_t i = 0; i <= m + n; ++i) {
      uint64_t a = 0, b = 0;
      for (uint64_t o = 0; o < i; ++o) {  // the merge's first i outputs
        const bool take_a = a < m && (b == n || (desc ? A[a] >= B[b] : A[a] <= B[b]));
        take_a ? ++a : ++b;
      }
      uint64_t j = 0, k = 0;
      CHECK(cm_co_rank_host(desc ? CM_KEY_U32_DESC : CM_KEY_U32, i, A.data(), m, B.data(), n, &j, &k) == CM_OK);
      CHECK(j == a && k == b);
    }
    uint64_t j, k;
    CHECK(cm_co_rank_host(0, m + n + 1, A.data(), m, B.data(), n, &j, &k) == CM_ERANGE);
  }
}

// The serving runtime: client threads submit (device-pointer and host
// requests), one thread polls and releases; every ticket is reported once.
static void server(int clients, int per_client) {
  const uint64_t arena_bytes = 64ull << 20;
  std::vector<uint64_t> arena(arena_bytes / 8);
  cm_server* s = nullptr;
  CHECK(cm_server_create(0, 1, arena.data(), arena_bytes, 8, 2, 256, &s) == CM_OK);
  if (!s) return;
  const uint64_t total = (uint64_t)clients * per_client;
  std::atomic<uint64_t> submitted{0};
  std::mutex mu;
  // tickets the clients got back, and tickets the poller saw reported (a
  // report can come before its client has recorded the ticket)
  std::set<uint64_t> tickets, reported_set;
  std::vector<std::thread> th;
  for (int c = 0; c < clients; ++c) {
    th.emplace_back([&, c] {
      std::mt19937_64 rng(100 + c);
      std::vector<uint32_t> keys(1 << 16), vals(1 << 16), out_k(1 << 17), out_v(1 << 17);
      for (int r = 0; r < per_client; ++r) {
        const uint64_t m = rng() % 5000, n = rng() % 5000;
        uint64_t t = 0;
        int rc;
        do {
          if (r % 3 == 2)  // host request: staged in the arena and copied back
            rc = cm_server_submit_host(s, keys.data(), vals.data(), m, keys.data() + 8192, vals.data() + 8192, n,
                                       out_k.data(), out_v.data(), &t);
          else
            rc = cm_server_submit(s, keys.data(), vals.data(), m, keys.data() + 8192, vals.data() + 8192, n, nullptr,
                                  r % 3 == 1, &t);
          if (rc == CM_EBUSY) std::this_thread::yield();
        } while (rc == CM_EBUSY);
        CHECK(rc == CM_OK);
        {
          std::lock_guard<std::mutex> lk(mu);
          CHECK(tickets.insert(t).second);
        }
        ++submitted;
        // a host request's arrays stay alive and untouched until it is
        // reported: wait for that before reusing them
        if (r % 3 == 2) {
          for (;;) {
            std::lock_guard<std::mutex> lk(mu);
            if (reported_set.count(t)) break;
          }
        }
      }
    });
  }
  uint64_t reported = 0;
  cm_server_done done[32];
  while (reported < total) {
    uint32_t k = 0;
    CHECK(cm_server_poll(s, done, 32, &k, 1000) == CM_OK);
    for (uint32_t x = 0; x < k; ++x) {
      CHECK(done[x].status == CM_OK);
      CHECK(done[x].latency_ns >= done[x].ended_ns && done[x].ended_ns >= done[x].queued_ns);
      CHECK(cm_server_release(s, done[x].ticket) == CM_OK);
      CHECK(cm_server_release(s, done[x].ticket) == CM_EINVAL);  // released once only
      std::lock_guard<std::mutex> lk(mu);
      CHECK(reported_set.insert(done[x].ticket).second);  // reported once
    }
    reported += k;
  }
  for (auto& t : th) t.join();
  CHECK(tickets == reported_set && tickets.size() == total);
  cm_server_stats st;
  CHECK(cm_server_get_stats(s, &st) == CM_OK);
  CHECK(st.submitted == total && st.completed == total && st.failed == 0);
  CHECK(st.arena_peak_bytes <= arena_bytes);
  CHECK(cm_server_destroy(s) == CM_OK);
  printf("server: %llu requests from %d client threads reported once each in %llu batches\n",
         (unsigned long long)reported, clients, (unsigned long long)st.batches);

  // shutdown with requests that can never be admitted (the arena is held by
  // an unreleased output): they are cancelled
  CHECK(cm_server_create(0, 1, arena.data(), 1 << 20, 4, 1, 16, &s) == CM_OK);
  std::vector<uint32_t> keys(1 << 16), vals(1 << 16);
  uint64_t t1 = 0, t2 = 0;
  CHECK(cm_server_submit(s, keys.data(), vals.data(), 30000, keys.data(), vals.data(), 30000, nullptr, 0, &t1) ==
        CM_OK);
  uint32_t k = 0;
  while (k == 0) CHECK(cm_server_poll(s, done, 1, &k, 1000) == CM_OK);
  // 640 KB of outputs: more than the 1 MiB arena has left while the first
  // request's 480 KB are held
  CHECK(cm_server_submit(s, keys.data(), vals.data(), 40000, keys.data(), vals.data(), 40000, nullptr, 0, &t2) ==
        CM_OK);
  CHECK(cm_server_destroy(s) == CM_OK);
}

int main(int argc, char** argv) {
  const bool threads_only = argc > 1 && strcmp(argv[1], "threads") == 0;
  if (!threads_only) {
    abi_calls();
    host_co_rank();
    server(4, 60);
  } else {
    server(6, 150);
  }
  printf("host driver: %d failed checks\n", g_failures);
  return g_failures ? 1 : 0;
}

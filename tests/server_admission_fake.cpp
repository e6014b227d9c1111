// Fake executor for the server's memory admission: queries with random
// table sizes arrive and run for random numbers of steps; each step admits
// with srv::admit_fifo exactly as the server does.  Checks, at every step:
// the ranges out never overlap, never leave the pool and never sum above
// it; admission keeps submission order; every query that fits the pool is
// admitted in the end; the pool is whole again when all have finished.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <vector>

#include "../paper_2106_03058_amd/csrc/server_admission.h"

using agp::srv::RangePool;

static int fail(const char* what, long step) {
  std::printf("FAIL %s at step %ld\n", what, step);
  return 1;
}

int main(int argc, char** argv) {
  const unsigned seed = argc > 1 ? static_cast<unsigned>(std::atoi(argv[1])) : 1u;
  std::mt19937_64 rng(seed);
  const uint64_t pool_size = 1u << 20;
  const int slots = 48;
  const int nq = 4000;
  RangePool pool(pool_size);
  struct Q {
    uint64_t need, off = 0;
    int steps_left = 0;
    bool running = false, done = false, rejected = false;
  };
  std::vector<Q> q(nq);
  for (auto& x : q) {  // table sizes as the server makes them: powers of two, a few beyond the pool
    const double touched = std::exp(std::uniform_real_distribution<double>(2.0, 12.5)(rng));
    x.need = agp::srv::table_entries(touched, 1 << 22, 256);
    if (rng() % 97 == 0) x.need = pool_size * 2;
    x.steps_left = 1 + static_cast<int>(rng() % 40);
  }
  std::deque<uint64_t> pending;
  std::vector<uint64_t> order;  // admission order
  int next = 0, running = 0;
  long step = 0;
  for (; step < 1000000 && (next < nq || !pending.empty() || running > 0); ++step) {
    const int arrive = static_cast<int>(rng() % 6);
    for (int k = 0; k < arrive && next < nq; ++k) pending.push_back(static_cast<uint64_t>(next++));
    const bool gate_open = rng() % 8 != 0;  // now and then a work budget holds the head back
    agp::srv::admit_fifo(
        pending, slots - running, pool, [&](uint64_t t) { return q[t].need; },
        [&](uint64_t) { return gate_open; },
        [&](uint64_t t, uint64_t off) {
          q[t].off = off;
          q[t].running = true;
          ++running;
          order.push_back(t);
        },
        [&](uint64_t t) {
          q[t].rejected = true;
          order.push_back(t);
        });
    // invariants over the running queries
    uint64_t sum = 0;
    std::vector<std::pair<uint64_t, uint64_t>> rs;
    for (const auto& x : q)
      if (x.running) {
        sum += x.need;
        rs.emplace_back(x.off, x.need);
        if (x.off + x.need > pool_size) return fail("range outside the pool", step);
      }
    if (sum > pool_size) return fail("over-committed", step);
    if (sum != pool.used()) return fail("pool accounting", step);
    std::sort(rs.begin(), rs.end());
    for (size_t i = 1; i < rs.size(); ++i)
      if (rs[i - 1].first + rs[i - 1].second > rs[i].first) return fail("overlapping ranges", step);
    if (running > slots) return fail("more queries than slots", step);
    // one step of work; finished queries give their range back
    for (auto& x : q)
      if (x.running && --x.steps_left == 0) {
        pool.release(x.off, x.need);
        x.running = false;
        x.done = true;
        --running;
      }
  }
  for (size_t i = 1; i < order.size(); ++i)
    if (order[i] < order[i - 1]) return fail("admission out of submission order", step);
  int done = 0, rejected = 0;
  for (const auto& x : q) {
    if (x.need > pool_size) {
      if (!x.rejected) return fail("an oversized query was not rejected", step);
      ++rejected;
    } else if (!x.done) {
      return fail("a query that fits never finished", step);
    } else {
      ++done;
    }
  }
  if (pool.used() != 0 || pool.largest_free() != pool_size) return fail("pool not whole at the end", step);
  std::printf("ok %d done %d rejected %ld steps\n", done, rejected, step);
  return 0;
}

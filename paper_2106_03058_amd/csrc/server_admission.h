// Host-side memory admission of the query server (no device code): a
// first-fit pool of table entries that running queries borrow contiguous
// ranges from, and the size of a query's tables from its push estimate.
#pragma once

#include <cstdint>
#include <deque>
#include <iterator>
#include <map>

namespace agp {
namespace srv {

// Contiguous ranges [off, off + len) of a pool of `size` entries, handed out
// first fit (lowest address) and coalesced when returned.  A range is never
// handed out twice, and the ranges out never exceed the pool.
class RangePool {
 public:
  explicit RangePool(uint64_t size = 0) { reset(size); }

  void reset(uint64_t size) {
    size_ = size;
    used_ = 0;
    free_.clear();
    if (size > 0) free_[0] = size;
  }

  bool alloc(uint64_t len, uint64_t* off) {
    if (len == 0) return false;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const uint64_t rest = it->second - len;
      const uint64_t at = it->first + len;
      free_.erase(it);
      if (rest > 0) free_[at] = rest;
      used_ += len;
      return true;
    }
    return false;
  }

  void release(uint64_t off, uint64_t len) {
    if (len == 0) return;
    used_ -= len;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + len == next->first) {  // merge with the range after
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {  // merge with the range before
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += len;
        return;
      }
    }
    free_[off] = len;
  }

  uint64_t size() const { return size_; }
  uint64_t used() const { return used_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& kv : free_) m = kv.second > m ? kv.second : m;
    return m;
  }
  const std::map<uint64_t, uint64_t>& free_ranges() const { return free_; }

 private:
  uint64_t size_ = 0;
  uint64_t used_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length, disjoint and not adjacent
};

// Entries of each of a query's two residue tables: a hashed table of a power
// of two at least twice the distinct nodes its busiest level is expected to
// touch (Theorem 3.3 bounds the expected pushes of each level, and a level
// touches at most as many nodes as it pushes to; at most half full, linear
// probing stays short), at least min_entries; or, when that would reach n,
// a direct table of exactly n entries (position = node).
inline uint64_t table_entries(double touched, int64_t n, uint64_t min_entries = 256) {
  const uint64_t nn = static_cast<uint64_t>(n > 0 ? n : 1);
  if (!(touched < static_cast<double>(nn))) return nn;
  uint64_t e = min_entries;
  while (static_cast<double>(e) < 2.0 * touched && e < nn) e <<= 1;
  return e < nn ? e : nn;
}

// One admission round, in submission order: while a slot is free and the
// query at the head of the queue gets a range of its table entries, admit it
// (on_admit(ticket, offset)); a query that needs more than the whole pool is
// rejected (on_reject(ticket)) and the next one considered; a query that
// does not fit now, or that may_admit(ticket) holds back (a work budget),
// waits at the head, and so does everything behind it.  Returns the number
// admitted.
template <class Need, class MayAdmit, class OnAdmit, class OnReject>
int admit_fifo(std::deque<uint64_t>& pending, int free_slots, RangePool& pool, Need need, MayAdmit may_admit,
               OnAdmit on_admit, OnReject on_reject) {
  int admitted = 0;
  while (free_slots > 0 && !pending.empty()) {
    const uint64_t t = pending.front();
    const uint64_t len = need(t);
    if (len > pool.size()) {
      pending.pop_front();
      on_reject(t);
      continue;
    }
    if (!may_admit(t)) break;
    uint64_t off = 0;
    if (!pool.alloc(len, &off)) break;
    pending.pop_front();
    on_admit(t, off);
    --free_slots;
    ++admitted;
  }
  return admitted;
}

}  // namespace srv
}  // namespace agp

// Work lists of active tree nodes, built by the whole GPU. A list is a sequence of passes,
// each one tree level with a filter on the node's split flag, over the Morton codes of that
// level's node grid (Morton order keeps neighbouring nodes close in the list). Blocks take
// kCodesPerBlock consecutive codes of one pass: a first kernel counts the nodes each block
// keeps, a one-block-per-scan kernel turns the counts into offsets (and per-slot totals),
// and a third kernel writes the items in code order. The list is the same as one built
// sequentially pass by pass.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wamct {
namespace {

constexpr int kMaxPasses = 16;
constexpr int kListThreads = 1024;
constexpr int kListRounds = 4;
constexpr int kCodesPerBlock = kListRounds * kListThreads;

struct PassTable {
  int n_pass;
  int level[kMaxPasses];
  int filter[kMaxPasses];          // 0: split nodes only, 1: unsplit nodes only, 2: every node
  int slot[kMaxPasses];            // count slot (index into the scan's counts) the pass adds to
  int n_slot;                      // slots 1 .. n_slot are written; slot 0 gets the total
  int64_t total[kMaxPasses];       // Morton codes of the pass
  int blk_start[kMaxPasses + 1];   // first block of each pass; blk_start[n_pass] = blocks per scan
};

// Appends a pass over `codes` Morton codes; returns false when the table is full.
inline bool add_pass(PassTable& pt, int level, int filter, int slot, int64_t codes) {
  if (pt.n_pass >= kMaxPasses) return false;
  const int p = pt.n_pass++;
  pt.level[p] = level;
  pt.filter[p] = filter;
  pt.slot[p] = slot;
  pt.total[p] = codes;
  pt.blk_start[p + 1] = pt.blk_start[p] + int((codes + kCodesPerBlock - 1) / kCodesPerBlock);
  if (slot > pt.n_slot) pt.n_slot = slot;
  return true;
}

__device__ inline int pass_of(const PassTable& pt, int b) {
  int p = 0;
  while (p + 1 < pt.n_pass && pt.blk_start[p + 1] <= b) ++p;
  return p;
}

// Spec::keep(scan, level, filter, code, word) -> whether the node of Morton code `code` at
// `level` is in the list (and its item word).
template <class Spec>
__global__ __launch_bounds__(kListThreads) void k_list_count(Spec sp, PassTable pt, int* __restrict__ bcount) {
  __shared__ int wt[kListThreads / 64];
  const int b = blockIdx.x, scan = blockIdx.y, nblk = pt.blk_start[pt.n_pass];
  const int p = pass_of(pt, b);
  const int64_t c0 = int64_t(b - pt.blk_start[p]) * kCodesPerBlock;
  int cnt = 0;   // wave-uniform
  for (int r = 0; r < kListRounds; ++r) {
    const int64_t code = c0 + r * kListThreads + threadIdx.x;
    uint32_t word = 0;
    const bool keep = code < pt.total[p] && sp.keep(scan, pt.level[p], pt.filter[p], code, word);
    cnt += __popcll(__ballot(keep));
  }
  if ((threadIdx.x & 63) == 0) wt[threadIdx.x >> 6] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < kListThreads / 64; ++w) t += wt[w];
    bcount[int64_t(scan) * nblk + b] = t;
  }
}

// One block per scan: exclusive offsets of the blocks, per-slot totals into counts[slot]
// and the list length into counts[0] (counts of scan p at counts + p cstride).
__global__ __launch_bounds__(kListThreads) void k_list_scan(PassTable pt, const int* __restrict__ bcount,
                                                            int* __restrict__ boff, int* __restrict__ counts,
                                                            int cstride) {
  __shared__ int wsum[kListThreads / 64];
  __shared__ int pass_cnt[kMaxPasses];
  const int scan = blockIdx.x, nblk = pt.blk_start[pt.n_pass];
  bcount += int64_t(scan) * nblk;
  boff += int64_t(scan) * nblk;
  counts += int64_t(scan) * cstride;
  if (threadIdx.x < kMaxPasses) pass_cnt[threadIdx.x] = 0;
  const int per = (nblk + kListThreads - 1) / kListThreads;
  const int b0 = min(nblk, int(threadIdx.x) * per), b1 = min(nblk, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += bcount[b];
  // exclusive scan of the per-thread sums: within each wave by shuffles, then over waves
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int v = s;
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  if (lane == 63) wsum[wv] = v;
  __syncthreads();
  int acc = v - s;
  for (int w = 0; w < wv; ++w) acc += wsum[w];
  int p = b0 < nblk ? pass_of(pt, b0) : 0, run = 0;
  for (int b = b0; b < b1; ++b) {
    while (pt.blk_start[p + 1] <= b) {   // block b belongs to a later pass
      if (run) atomicAdd(&pass_cnt[p], run);
      run = 0;
      ++p;
    }
    const int c = bcount[b];
    boff[b] = acc;
    acc += c;
    run += c;
  }
  if (run) atomicAdd(&pass_cnt[p], run);
  __syncthreads();
  if (threadIdx.x == 0) {
    int tot = 0;
    for (int k = 1; k <= pt.n_slot; ++k) counts[k] = 0;
    for (int q = 0; q < pt.n_pass; ++q) {
      counts[pt.slot[q]] += pass_cnt[q];
      tot += pass_cnt[q];
    }
    counts[0] = tot;
  }
}

// Writes each block's kept items from its offset, in code order (items of scan p at
// items + p istride).
template <class Spec>
__global__ __launch_bounds__(kListThreads) void k_list_write(Spec sp, PassTable pt, const int* __restrict__ boff,
                                                             uint32_t* __restrict__ items, int64_t istride) {
  __shared__ int wt[kListThreads / 64];
  const int b = blockIdx.x, scan = blockIdx.y, nblk = pt.blk_start[pt.n_pass];
  const int p = pass_of(pt, b);
  const int64_t c0 = int64_t(b - pt.blk_start[p]) * kCodesPerBlock;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  items += int64_t(scan) * istride;
  int base = boff[int64_t(scan) * nblk + b];
  for (int r = 0; r < kListRounds; ++r) {
    const int64_t code = c0 + r * kListThreads + threadIdx.x;
    uint32_t word = 0;
    const bool keep = code < pt.total[p] && sp.keep(scan, pt.level[p], pt.filter[p], code, word);
    const uint64_t bal = __ballot(keep);
    if (lane == 0) wt[wv] = __popcll(bal);
    __syncthreads();
    int off = base, all = 0;
    for (int w = 0; w < kListThreads / 64; ++w) {
      if (w < wv) off += wt[w];
      all += wt[w];
    }
    if (keep) items[off + __popcll(bal & ((uint64_t(1) << lane) - 1))] = word;
    base += all;
    __syncthreads();
  }
}

}  // namespace
}  // namespace wamct

// On-device k-th smallest selection (MSB-first radix select, 4 passes of 8
// bits over an order-preserving uint32 image of the float keys) for several
// segments at once.  Used for the nearest-rank percentiles of the loss weight
// (Sec. IV-B) and for the per-bin quantile cutoffs and depth percentiles
// (Sec. IV-C).  Exact: the result is an element of the segment.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lv {

// Block histograms are spread over lane-indexed copies, padded so that the
// copies of one bin fall in different LDS banks.
constexpr int kHistCopies = 16;
constexpr int kHistStride = 257;

struct SelState {
  uint32_t prefix;  // decided high bits of the answer's key
  uint32_t k;       // rank (0-based) still to find among keys matching prefix
  uint32_t n;       // segment size
  uint32_t valid;   // 0: empty segment, no answer
};

__device__ __forceinline__ uint32_t f2key(float f) {
  const uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__device__ __forceinline__ float key2f(uint32_t k) {
  const uint32_t u = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
  return __uint_as_float(u);
}

__device__ __forceinline__ int sel_shift(int pass) { return 24 - 8 * pass; }
__device__ __forceinline__ uint32_t sel_himask(int pass) {
  return pass == 0 ? 0u : (0xFFFFFFFFu << (sel_shift(pass) + 8));
}

// nseg simultaneous selections.  hist[4][nseg][256] holds the digit counts
// of each pass (zero before its pass); st[2][nseg] holds each segment's state
// after an even (row 0) or odd (row 1) number of passes.  There is no
// separate digit-choice launch: the launch that needs the state before pass p
// (pass p's histogram, or the consumer with p = 4) chooses pass p-1's digit
// itself from that pass's complete histogram, every block redundantly, and
// block 0 stores the result in row p & 1 for the next launch.  It reads row
// (p-1) & 1, so no block reads a state while another overwrites it.
struct SelSet {
  SelState* st;
  uint32_t* hist;
  int nseg;
};

__device__ __forceinline__ uint32_t* sel_hist(const SelSet& S, int pass, int sg) {
  return S.hist + (size_t(pass) * size_t(S.nseg) + size_t(sg)) * 256;
}

// Digit choice of one pass for one segment, by one full wave (each lane
// holds 4 consecutive bins): the digit whose cumulative count passes k joins
// the prefix and k drops by the counts before it.  A segment with no answer
// is returned unchanged.
__device__ __forceinline__ SelState sel_advance(SelState s, const uint32_t* h, int pass) {
  const int lane = threadIdx.x & 63;
  const uint4 c4 = *reinterpret_cast<const uint4*>(h + 4 * lane);
  const uint32_t c[4] = {c4.x, c4.y, c4.z, c4.w};
  const uint32_t tot = (c[0] + c[1]) + (c[2] + c[3]);
  uint32_t incl = tot;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  const uint32_t excl = incl - tot;
  const bool mine = s.valid != 0u && excl <= s.k && s.k < incl;   // the lane whose bins hold rank k
  uint32_t digit = 0u, below = excl;
  if (mine) {
    uint32_t d = 0u;
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j) {
      if (d == j && s.k >= below + c[j]) {
        below += c[j];
        d = j + 1u;
      }
    }
    digit = 4u * uint32_t(lane) + d;
  }
  const unsigned long long b = __ballot(mine);
  if (b != 0ull) {
    const int src = __builtin_ctzll(b);
    digit = uint32_t(__shfl(int(digit), src, 64));
    below = uint32_t(__shfl(int(below), src, 64));
    s.prefix |= digit << sel_shift(pass);
    s.k -= below;
  }
  return s;
}

// State of segment sg before pass `pass` (0..3; 4 = the answer), by one full
// wave.  Pass 0 reads the initial state.
__device__ __forceinline__ SelState sel_state(const SelSet& S, int sg, int pass) {
  if (pass == 0) return S.st[sg];
  return sel_advance(S.st[size_t((pass - 1) & 1) * size_t(S.nseg) + size_t(sg)], sel_hist(S, pass - 1, sg),
                     pass - 1);
}

// block 0 of a launch, one lane: keep the state for the next launch
__device__ __forceinline__ void sel_store(const SelSet& S, int sg, int pass, const SelState& s) {
  S.st[size_t(pass & 1) * size_t(S.nseg) + size_t(sg)] = s;
}

// ------------------------------------------------------- capped selection
// Of the candidates among n items, marks the first min(cap, #candidates) in
// the order (key, index): an exact radix select of the cap-th smallest key
// among the candidates, then the candidates equal to it taken in index order
// (block-ordered count).  A producer kernel with at most kCapFillBlocks
// blocks writes key[i] and cand[i] for every item and its block's candidate
// count with cap_store_block_count; launch_cap_setup must run before it.
constexpr int kCapFillBlocks = 1024;

// constants of the subdivision selection (eq. 13-16)
struct SplitParams {
  float kappa, beta;
  uint32_t max_splits;
};

constexpr int kCapHistBlocks = 256;
constexpr int kCapPer = 2048;   // items per block of the block-ordered passes

struct CapWS {
  uint32_t* key;     // [n]
  uint8_t* cand;     // [n]
  uint32_t* ublk;    // [kCapFillBlocks] candidates per producer block
  uint32_t* eqblk;   // [ceil(n / kCapPer)] candidates equal to the cutoff per block
  uint32_t* cnt;     // [0]: candidates
  SelSet sel;        // one selection: hist [4][256], st [2]
};

uint64_t cap_ws_bytes(int64_t n);
CapWS cap_bind(void* base, int64_t n);
hipError_t launch_cap_setup(const CapWS& w, uint32_t* count_out, hipStream_t s);
// mask[i] = 1 for the marked items, else 0; count_out (nullable) = how many
hipError_t launch_cap_select(const CapWS& w, int64_t n, uint32_t cap, uint8_t* mask,
                             uint32_t* count_out, hipStream_t s);

// block-wide sum of the calling threads' candidate counts into ublk
// (every thread of the block must call it)
__device__ __forceinline__ void cap_store_block_count(const CapWS& w, uint32_t mine) {
  __shared__ uint32_t s_c[32];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mine += uint32_t(__shfl_xor(int(mine), o, 64));
  if ((threadIdx.x & 63) == 0) s_c[threadIdx.x >> 6] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t k = 0; k < (blockDim.x + 63) / 64; ++k) t += s_c[k];
    w.ublk[blockIdx.x] = t;
  }
}

}  // namespace lv

// Fused multi-gate passes: one HBM read and one write of the state for a run
// of consecutive gates (Op1/Op2/Op3 of §3a-§3c applied in circuit order).
//
// A pass picks T "tile bits": the lowest L bits of the label (so a tile is
// made of contiguous 2^L-amplitude chunks and loads stay coalesced) plus the
// target bits of every gate in the run.  The state splits into 2^(nq-T)
// tiles, one per value of the other bits; every gate of the run touches only
// tile bits, so each tile can be loaded into LDS, advanced through the whole
// run, and stored back, independently of all other tiles.  Inside the tile a
// gate is the same group update as the one-gate sweep (same member order, same
// FMA sequence), so the results equal the one-sweep-per-gate path bit for bit.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "qcw_device.h"
#include "qcw_host.h"

namespace qcw {

constexpr int kFusedMaxFree = 10;  // tile bits above the contiguous low bits
constexpr int kFusedDefaultTile = 12;
constexpr int kFusedDefaultLow = 4;
constexpr int kFuseExtraFlops = 2;  // see plan_passes

// Threads per block for a tile of 2^T amplitudes: eight amplitudes per thread
// from T = 11 up, so larger tiles also get more waves for their gates.
constexpr int fused_block(int T) { return T <= 11 ? 256 : (1 << (T - 3)); }

struct alignas(16) FusedGate {
  int32_t k;
  int32_t sb0, sb1, sb2;  // local (tile-index) target bits, ascending
  int32_t m3;             // 0: u is U; 1: three-product form (u = (A, -(A+B)), d = B - A)
  int32_t pad[3];
  uint32_t off[8];        // local member offsets, local index order
  double2 u[64];          // m x m, row-major (see m3)
  double d[64];           // m x m, row-major, three-product form only
};

struct alignas(16) FusedPass {
  int32_t ngates;
  int32_t gate_off;        // first gate in the gate table
  int32_t T, L;            // tile bits, contiguous low bits
  int32_t n_outer;         // number of non-tile bits
  int32_t pad[3];
  uint64_t chunk_off[1 << kFusedMaxFree];  // label offset of chunk c within the tile
  uint8_t outer_pos[40];   // positions of the non-tile bits, ascending
};

typedef double v2d __attribute__((ext_vector_type(2)));

// Wave chunks.  A block of NT threads has NT / 64 waves; the tile bits below
// wave_tile_bits<T, NT> index within a chunk of the tile, the bits above
// pick the chunk.  A gate whose targets are all below that bit maps every
// chunk onto itself: when each wave takes its groups from its own chunk, two
// such gates in a row need no block barrier between them (a wave's LDS
// operations complete in order), and neither do the staging of the tile and
// such a gate, done chunk by chunk as well.
template <int T, int NT>
constexpr int wave_tile_bits() {
  return T - (NT >= 1024 ? 4 : NT >= 512 ? 3 : NT >= 256 ? 2 : NT >= 128 ? 1 : 0);
}

// Group i of thread tid for a K-qubit gate: strided over the block, or
// (local) within the thread's wave chunk.  Either way the groups of a gate
// are dealt out once each, and each is computed as in the sweep.
template <int K, int NT, int T>
__device__ __forceinline__ uint32_t group_of(int i, uint32_t tid, bool local) {
  constexpr int TW = wave_tile_bits<T, NT>();
  if (TW - K >= 6 && local)
    return ((tid >> 6) << (TW - K)) | ((uint32_t)i << 6) | (tid & 63u);
  return (uint32_t)i * NT + tid;
}

// The gate keeps every wave chunk (all targets below the chunk bits), and
// its groups fill whole waves (so group_of may deal them per chunk).
template <int T, int NT>
__device__ __forceinline__ bool chunk_local(const FusedGate &g) {
  constexpr int TW = wave_tile_bits<T, NT>();
  const int top = g.k == 1 ? g.sb0 : g.k == 2 ? g.sb1 : g.sb2;
  return top < TW && TW - g.k >= 6;
}

// One gate on a tile of 2^T amplitudes in LDS, NT threads.  Each thread owns
// 2^(T-K) / NT groups (fixed at compile time) and issues the LDS reads of all
// of them before any arithmetic, so several reads are in flight per lane.
template <int K, int NT, int T>
__device__ __forceinline__ void tile_gate(double2 *S, const FusedGate &g, bool local) {
  constexpr int M = 1 << K;
  constexpr uint32_t NG = 1u << (T - K);
  constexpr int G = NG >= NT ? (int)(NG / NT) : 1;
  const uint32_t tid = threadIdx.x % NT;
  double2 x[G][M];
  uint32_t base[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint32_t j = group_of<K, NT, T>(i, tid, local);
    base[i] = insert_zeros<K, uint32_t>(j, g.sb0, g.sb1, g.sb2);
    if (NG >= NT || j < NG) {
#pragma unroll
      for (int r = 0; r < M; ++r) x[i][r] = S[base[i] + g.off[r]];
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint32_t j = group_of<K, NT, T>(i, tid, local);
    if (NG >= NT || j < NG) {
      const uint32_t b = base[i];
      group_matvec_put<M>(x[i], [&](int r, int c) { return g.u[r * M + c]; },
                          [&](int r, double2 y) { S[b + g.off[r]] = y; });
    }
  }
}

// The same gate in the three-product form (U = A + iB on x = a + ib):
//   Re y = A (a + b) - (A + B) b,   Im y = A (a + b) + (B - A) a,
// with A + B and B - A formed on the host: per output row one shared real
// product A (a + b) and one more real product for each part, 3m FMAs instead
// of 4m (plus m additions for a + b per group).  The rounding differs from
// the direct product (each term is bounded by a small multiple of |U| |x|, so
// the error stays within a small factor of it).
template <int K, int NT, int T>
__device__ __forceinline__ void tile_gate3m(double2 *S, const FusedGate &g, bool local) {
  constexpr int M = 1 << K;
  constexpr uint32_t NG = 1u << (T - K);
  constexpr int G = NG >= NT ? (int)(NG / NT) : 1;
  const uint32_t tid = threadIdx.x % NT;
  double2 x[G][M];
  uint32_t base[G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint32_t j = group_of<K, NT, T>(i, tid, local);
    base[i] = insert_zeros<K, uint32_t>(j, g.sb0, g.sb1, g.sb2);
    if (NG >= NT || j < NG) {
#pragma unroll
      for (int r = 0; r < M; ++r) x[i][r] = S[base[i] + g.off[r]];
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const uint32_t j = group_of<K, NT, T>(i, tid, local);
    if (NG >= NT || j < NG) {
      double sum[M];
#pragma unroll
      for (int c = 0; c < M; ++c) sum[c] = x[i][c].x + x[i][c].y;
#pragma unroll
      for (int r = 0; r < M; ++r) {
        double t = 0.0;
#pragma unroll
        for (int c = 0; c < M; ++c) t = __fma_rn(g.u[r * M + c].x, sum[c], t);
        double re = t, im = t;
#pragma unroll
        for (int c = 0; c < M; ++c) re = __fma_rn(g.u[r * M + c].y, x[i][c].y, re);
#pragma unroll
        for (int c = 0; c < M; ++c) im = __fma_rn(g.d[r * M + c], x[i][c].x, im);
        S[base[i] + g.off[r]] = make_double2(re, im);
      }
    }
  }
}

// One gate of a pass on a tile, in the form its plan chose.
template <int NT, int T>
__device__ __forceinline__ void tile_apply(double2 *S, const FusedGate &g, bool local = false) {
  if (g.m3) {
    switch (g.k) {
      case 1: tile_gate3m<1, NT, T>(S, g, local); break;
      case 2: tile_gate3m<2, NT, T>(S, g, local); break;
      default: tile_gate3m<3, NT, T>(S, g, local); break;
    }
  } else {
    switch (g.k) {
      case 1: tile_gate<1, NT, T>(S, g, local); break;
      case 2: tile_gate<2, NT, T>(S, g, local); break;
      default: tile_gate<3, NT, T>(S, g, local); break;
    }
  }
}

// Each thread stages 2^T / NT amplitudes of the tile.
template <int T, int L, int NT = fused_block(T)>
__global__ __launch_bounds__(NT) void fused_pass_kernel(double2 *psi,
                                                                 const FusedPass *__restrict__ passes,
                                                                 const FusedGate *__restrict__ gates,
                                                                 int p) {
  extern __shared__ double2 S[];
  constexpr int N_TILE = 1 << T;
  constexpr int PER = N_TILE / NT;
  const FusedPass &P = passes[p];
  // Label of the tile's first amplitude: block index bits deposited at the
  // non-tile bit positions.
  uint64_t tile_base = 0;
  {
    uint64_t b = blockIdx.x;
    for (int j = 0; j < P.n_outer; ++j) tile_base |= ((b >> j) & 1ull) << P.outer_pos[j];
  }
  // Amplitude q of this thread: element q * 64 + lane of its wave's chunk
  // (64 consecutive elements per wave and q: whole 16-amplitude chunks of
  // the state, as before).
  constexpr int TW = wave_tile_bits<T, NT>();
  static_assert(PER == 1 << (TW - 6), "a wave chunk is PER elements per lane");
  const uint32_t chunk0 = (threadIdx.x >> 6) << TW, lane = threadIdx.x & 63u;
  v2d v[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = chunk0 | ((uint32_t)q << 6) | lane;
    const uint64_t lab = tile_base + P.chunk_off[i >> L] + (uint32_t)(i & ((1 << L) - 1));
    v[q] = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(psi + lab));
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) S[chunk0 | ((uint32_t)q << 6) | lane] = make_double2(v[q].x, v[q].y);
  // A block barrier separates two steps unless both keep every wave in its
  // chunk (the staging and the store do).
  bool prev_local = true;
  for (int gi = 0; gi < P.ngates; ++gi) {
    const FusedGate &g = gates[P.gate_off + gi];
    const bool local = chunk_local<T, NT>(g);
    if (!(local && prev_local)) __syncthreads();
    tile_apply<NT, T>(S, g, local);
    prev_local = local;
  }
  if (!prev_local) __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const uint32_t i = chunk0 | ((uint32_t)q << 6) | lane;
    const uint64_t lab = tile_base + P.chunk_off[i >> L] + (uint32_t)(i & ((1 << L) - 1));
    const double2 a = S[i];
    v2d w = {a.x, a.y};
    __builtin_nontemporal_store(w, reinterpret_cast<v2d *>(psi + lab));
  }
}

// Persistent, software-pipelined form for large tiles (one or two blocks per
// CU): each block walks tiles blockIdx.x, blockIdx.x + gridDim.x, ...; the
// global loads of the next tile are issued into registers before the current
// tile's gates run in LDS, so HBM reads overlap the LDS work and the stores.
template <int T, int L, int NT = fused_block(T)>
__global__ __launch_bounds__(NT) void fused_persistent_kernel(double2 *psi,
                                                              const FusedPass *__restrict__ passes,
                                                              const FusedGate *__restrict__ gates,
                                                              int p, uint64_t ntiles) {
  extern __shared__ double2 S[];
  constexpr int PER = (1 << T) / NT;
  const FusedPass &P = passes[p];
  auto base_of = [&](uint64_t t) {
    uint64_t b = 0;
    for (int j = 0; j < P.n_outer; ++j) b |= ((t >> j) & 1ull) << P.outer_pos[j];
    return b;
  };
  uint64_t lab[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int i = q * NT + threadIdx.x;
    lab[q] = P.chunk_off[i >> L] + (uint32_t)(i & ((1 << L) - 1));
  }
  uint64_t t = blockIdx.x;
  if (t >= ntiles) return;
  v2d v[PER];
  uint64_t base = base_of(t);
#pragma unroll
  for (int q = 0; q < PER; ++q)
    v[q] = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(psi + base + lab[q]));
  for (;;) {
#pragma unroll
    for (int q = 0; q < PER; ++q) S[q * NT + threadIdx.x] = make_double2(v[q].x, v[q].y);
    __syncthreads();
    const uint64_t tn = t + gridDim.x;
    const bool more = tn < ntiles;
    const uint64_t base_n = more ? base_of(tn) : 0;
    if (more) {
#pragma unroll
      for (int q = 0; q < PER; ++q)
        v[q] = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(psi + base_n + lab[q]));
    }
    for (int gi = 0; gi < P.ngates; ++gi) {
      const FusedGate &g = gates[P.gate_off + gi];
      tile_apply<NT, T>(S, g);
      __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const double2 a = S[q * NT + threadIdx.x];
      v2d w = {a.x, a.y};
      __builtin_nontemporal_store(w, reinterpret_cast<v2d *>(psi + base + lab[q]));
    }
    if (!more) break;
    __syncthreads();  // every thread has read its part of S before it is refilled
    t = tn;
    base = base_n;
  }
}

// LDS-only block barrier: waits for this wave's LDS operations, then the
// workgroup barrier.  Outstanding global loads stay in flight across it (a
// full __syncthreads would also wait for them).  The memory clobber keeps the
// compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Warp-specialised persistent pass for 2^12-amplitude tiles: 1024 threads per
// block, one block per CU, two LDS tile buffers.  Threads 0..511 apply the
// run of gates to the tile in one buffer; threads 512..1023 meanwhile store
// the previous tile from the other buffer and load the next tile into it.
// Both halves pass the same barriers (one per gate); the loading half writes
// its registers into LDS only in the last gate interval, so its loads are in
// flight during the whole compute phase.
template <int L>
__global__ __launch_bounds__(1024) void fused_ws_kernel(double2 *psi,
                                                        const FusedPass *__restrict__ passes,
                                                        const FusedGate *__restrict__ gates,
                                                        int p, uint64_t ntiles) {
  constexpr int T = 12;
  constexpr int NC = 512;                 // compute threads
  constexpr int PER = (1 << T) / 512;     // amplitudes per memory thread
  extern __shared__ double2 S2[];
  const FusedPass &P = passes[p];
  const bool mem = threadIdx.x >= NC;
  const int tm = threadIdx.x - NC;        // memory-thread index (valid when mem)
  // tiles of this block: blockIdx.x, blockIdx.x + gridDim.x, ...
  if ((uint64_t)blockIdx.x >= ntiles) return;
  const uint64_t n_it = (ntiles - 1 - blockIdx.x) / gridDim.x + 1;
  auto base_of = [&](uint64_t t) {
    uint64_t b = 0;
    for (int j = 0; j < P.n_outer; ++j) b |= ((t >> j) & 1ull) << P.outer_pos[j];
    return b;
  };
  uint64_t lab[PER];
  if (mem) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int i = q * 512 + tm;
      lab[q] = P.chunk_off[i >> L] + (uint32_t)(i & ((1 << L) - 1));
    }
  }
  const int ng = P.ngates;
  v2d w[PER];
  uint64_t base_next = 0;
  if (mem) {
    const uint64_t b0 = base_of(blockIdx.x);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      w[q] = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(psi + b0 + lab[q]));
      S2[q * 512 + tm] = make_double2(w[q].x, w[q].y);
    }
  }
  lds_barrier();
  uint64_t base_prev = 0, base_cur = base_of(blockIdx.x);
  for (uint64_t it = 0; it < n_it; ++it) {
    double2 *X = S2 + ((it & 1) << T);
    double2 *Y = S2 + (((it + 1) & 1) << T);
    const bool has_next = it + 1 < n_it;
    if (mem) {
      if (it > 0) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
          const double2 a = Y[q * 512 + tm];
          v2d o = {a.x, a.y};
          __builtin_nontemporal_store(o, reinterpret_cast<v2d *>(psi + base_prev + lab[q]));
        }
      }
      if (has_next) {
        base_next = base_of(blockIdx.x + (it + 1) * gridDim.x);
#pragma unroll
        for (int q = 0; q < PER; ++q)
          w[q] = __builtin_nontemporal_load(reinterpret_cast<const v2d *>(psi + base_next + lab[q]));
      }
    }
    for (int gi = 0; gi < ng; ++gi) {
      if (!mem) {
        const FusedGate &g = gates[P.gate_off + gi];
        tile_apply<NC, T>(X, g);
      } else if (gi == ng - 1 && has_next) {
#pragma unroll
        for (int q = 0; q < PER; ++q) Y[q * 512 + tm] = make_double2(w[q].x, w[q].y);
      }
      lds_barrier();
    }
    base_prev = base_cur;
    base_cur = base_next;
  }
  // the last tile, finished in buffer (n_it - 1) & 1
  if (mem) {
    const double2 *Z = S2 + (((n_it - 1) & 1) << T);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const double2 a = Z[q * 512 + tm];
      v2d o = {a.x, a.y};
      __builtin_nontemporal_store(o, reinterpret_cast<v2d *>(psi + base_prev + lab[q]));
    }
  }
}

// ------------------------------------------------------------------ planning
struct FusedShape {
  int T, L;
};

static int popcount64(uint64_t x) { return __builtin_popcountll(x); }

// Cuts the gate list into passes.  A pass's tile bits are the low L bits and
// the target bits of its gates (at most T); every pass is then widened with the
// lowest unused bits (larger contiguous chunks).
//
// By default a pass is a run of consecutive gates, extended while its bits
// fit, and results equal the one-sweep-per-gate path bit for bit.  Three plan
// flags trade that for less work; each leaves the circuit's operator
// unchanged and changes only the rounding:
// * QCW_PLAN_COMMUTE: a pass may take any gate of the front, i.e. any gate
//   not yet placed that shares no qubit with an earlier gate not yet placed.
//   Gates on disjoint qubits commute (the tensor structure of §2c), so moving
//   a front gate ahead of the unplaced gates before it is exact, and gates
//   that share a qubit keep their order.  Each step takes the front gate that
//   fits and adds the fewest new tile bits, which packs more gates per pass
//   than taking front gates in list order (10 passes instead of 11 for the
//   nq = 31 benchmark circuit; 17 in list order); for large states a small
//   search over the ties (FrontPlanner::search) trims about one pass more.
// * QCW_PLAN_FUSE: inside each pass, gates spanning at most three qubits are
//   merged into one gate (their matrix product, the first gate rightmost), so
//   the tile makes fewer LDS round trips.  Alone it merges runs of
//   consecutive gates; with QCW_PLAN_COMMUTE a gate may also join a block
//   ahead of gates of the pass it shares no qubit with.
// * QCW_PLAN_3M: the tile applies each gate in the three-product form
//   (tile_gate3m), 3m instead of 4m FMAs per amplitude.  A merge may add at
//   most kFuseExtraFlops flops per amplitude: two one-qubit gates, or two
//   two-qubit gates sharing a qubit, are merged; a one-qubit gate and a
//   disjoint two-qubit gate (44 -> 62 flops) are not, since the in-tile work
//   is bound by FP64 arithmetic about as much as by LDS traffic (measured
//   slower at nq = 31).
struct PlanRun {
  std::vector<int> g;  // gate indices, in execution order
  uint64_t mask;       // tile bits before widening
};

namespace {

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014): a fixed stream, so plans
// are deterministic.
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
};

// Planning with QCW_PLAN_COMMUTE.  A gate is in the front when no unplaced
// gate before it in the list shares a qubit with it; a pass repeatedly takes
// a front gate that fits its tile, preferring the one that adds the fewest
// new tile bits, until none fits.
struct FrontState {
  std::vector<char> placed;
  std::vector<int> rem;  // unplaced gates, list order
};

class FrontPlanner {
 public:
  FrontPlanner(const std::vector<uint64_t> &gm, int T, uint64_t low) : gm_(gm), T_(T), low_(low) {}

  FrontState start() const {
    FrontState s;
    s.placed.assign(gm_.size(), 0);
    s.rem.resize(gm_.size());
    for (size_t g = 0; g < gm_.size(); ++g) s.rem[g] = (int)g;
    return s;
  }

  // One pass, placing its gates in s.  Ties among the front gates that add
  // the fewest new bits (at least one) go to the earliest, or with rng to a
  // random one; a gate adding no new bit is always taken first.
  PlanRun pass(FrontState &s, SplitMix64 *rng) const {
    PlanRun cur{{}, low_};
    uint64_t all = 0;  // qubits of the unplaced gates: no gate beyond them is in the front
    for (int g : s.rem) all |= gm_[g];
    for (;;) {
      uint64_t blocked = 0;
      int best_new = 64, zero = -1;
      ties_.clear();
      for (int g : s.rem) {
        if (s.placed[g]) continue;
        if (!(gm_[g] & blocked) && popcount64(cur.mask | gm_[g]) <= T_) {
          const int nw = popcount64(gm_[g] & ~cur.mask);
          if (nw == 0) {
            zero = g;
            break;
          }
          if (nw < best_new) {
            best_new = nw;
            ties_.clear();
            ties_.push_back(g);
          } else if (nw == best_new && rng) {
            ties_.push_back(g);
          }
        }
        blocked |= gm_[g];
        if (blocked == all) break;
      }
      // the first unplaced gate is always in the front and fits an empty
      // pass (k + L <= T), so every pass places at least one gate
      const int pick = zero >= 0 ? zero
                       : ties_.empty() ? -1
                       : rng ? ties_[rng->next() % ties_.size()]
                             : ties_[0];
      if (pick < 0) break;
      s.placed[pick] = 1;
      cur.mask |= gm_[pick];
      cur.g.push_back(pick);
    }
    size_t w = 0;
    for (int g : s.rem)
      if (!s.placed[g]) s.rem[w++] = g;
    s.rem.resize(w);
    return cur;
  }

  // Greedy passes (no rng) that place everything left in s.
  std::vector<PlanRun> finish(FrontState s) const {
    std::vector<PlanRun> runs;
    while (!s.rem.empty()) runs.push_back(pass(s, nullptr));
    return runs;
  }

  // Plan built pass by pass: each pass is the best of `trials` candidates
  // (the greedy one and trials - 1 with random ties), scored by the greedy
  // completion's pass count (lookahead < 0) or by the gates placed after
  // `lookahead` more greedy passes.  Stops early once it cannot beat `bound`
  // passes (returns an empty plan then).
  std::vector<PlanRun> search(int trials, int lookahead, size_t bound, uint64_t seed) const {
    SplitMix64 rng{seed};
    FrontState s = start();
    std::vector<PlanRun> runs;
    while (!s.rem.empty()) {
      if (runs.size() + 1 >= bound) return {};
      FrontState best_s;
      PlanRun best_r;
      long best_score = 0;
      for (int t = 0; t < trials; ++t) {
        FrontState c = s;
        PlanRun r = pass(c, t ? &rng : nullptr);
        long score;
        if (lookahead < 0) {
          score = -(long)finish(c).size();
        } else {
          FrontState d = c;
          for (int i = 0; i < lookahead && !d.rem.empty(); ++i) pass(d, nullptr);
          score = -(long)d.rem.size();
        }
        if (t == 0 || score > best_score) {
          best_score = score;
          best_s = std::move(c);
          best_r = std::move(r);
        }
      }
      s = std::move(best_s);
      runs.push_back(std::move(best_r));
    }
    return runs;
  }

 private:
  const std::vector<uint64_t> &gm_;
  int T_;
  uint64_t low_;
  mutable std::vector<int> ties_;
};

// Search effort for the commute planner: only for states of at least
// kSearchMinQubits qubits, where one pass takes well over a millisecond and
// a plan is cached per stream, and for lists of at most kSearchMaxGates gates
// (kRolloutMaxGates for scoring by full greedy completion).  Measured on random
// 124-gate circuits at nq = 31: ~8% fewer passes than the greedy plan.
constexpr int kSearchMinQubits = 24;
constexpr int kSearchMaxGates = 2048;
constexpr int kRolloutMaxGates = 512;
constexpr int kSearchTrials = 16;

}  // namespace

static std::vector<PlanRun> plan_runs(int nq, const std::vector<Geom> &geo, FusedShape sh,
                                      bool commute) {
  const int T = std::min(sh.T, nq);
  const int L = std::min(sh.L, T);
  const uint64_t low = (L >= 64) ? ~0ull : ((1ull << L) - 1);
  const int ng = (int)geo.size();
  std::vector<uint64_t> gm(ng);
  for (int g = 0; g < ng; ++g) {
    uint64_t m = 0;
    for (int j = 0; j < geo[g].k; ++j) m |= 1ull << geo[g].bit[j];
    gm[g] = m;
  }
  std::vector<PlanRun> runs;
  if (!commute) {
    PlanRun cur{{}, low};
    for (int g = 0; g < ng; ++g) {
      if (popcount64(cur.mask | gm[g]) > T) {
        runs.push_back(std::move(cur));
        cur = PlanRun{{}, low};
      }
      cur.mask |= gm[g];
      cur.g.push_back(g);
    }
    if (!cur.g.empty()) runs.push_back(std::move(cur));
    return runs;
  }
  FrontPlanner fp(gm, T, low);
  runs = fp.finish(fp.start());
  if (nq >= kSearchMinQubits && ng <= kSearchMaxGates) {
    // a small portfolio of scoring rules; the plan with the fewest passes wins
    // (the earliest on ties)
    const int lookaheads[3] = {-1, 1, 2};
    for (int la : lookaheads) {
      if (la < 0 && ng > kRolloutMaxGates) continue;
      std::vector<PlanRun> r = fp.search(kSearchTrials, la, runs.size(), 0x51ed2701u + la);
      if (!r.empty() && r.size() < runs.size()) runs.swap(r);
    }
  }
  return runs;
}

static int plan_passes(int nq, const std::vector<Geom> &geo, const qcw_gate *gates,
                       const qcw_c64 *mats, FusedShape sh, int plan,
                       std::vector<FusedPass> &passes, std::vector<FusedGate> &fg) {
  const bool fuse = (plan & QCW_PLAN_FUSE) != 0;
  const int T = std::min(sh.T, nq);
  const int L = std::min(sh.L, T);
  const std::vector<PlanRun> runs = plan_runs(nq, geo, sh, (plan & QCW_PLAN_COMMUTE) != 0);
  passes.clear();
  fg.clear();
  for (size_t r = 0; r < runs.size(); ++r) {
    uint64_t mask = runs[r].mask;
    for (int b = 0; b < nq && popcount64(mask) < T; ++b) mask |= 1ull << b;
    FusedPass P;
    memset(&P, 0, sizeof P);
    P.gate_off = (int)fg.size();
    P.T = T;
    P.L = L;
    // local index of each tile bit, and the non-tile bit positions
    int local_of[64];
    int nl = 0, no = 0;
    for (int b = 0; b < nq; ++b) {
      if ((mask >> b) & 1) {
        local_of[b] = nl++;
      } else {
        local_of[b] = -1;
        P.outer_pos[no++] = (uint8_t)b;
      }
    }
    P.n_outer = no;
    // chunk c: its free (non-low) tile bits, deposited at their label positions
    int free_pos[kFusedMaxFree];
    int nf = 0;
    for (int b = L; b < nq; ++b)
      if ((mask >> b) & 1) free_pos[nf++] = b;
    if (nf != T - L || nf > kFusedMaxFree) return fail(QCW_EINVAL, "fused tile planning failed");
    for (int c = 0; c < (1 << nf); ++c) {
      uint64_t o = 0;
      for (int j = 0; j < nf; ++j)
        if ((c >> j) & 1) o |= 1ull << free_pos[j];
      P.chunk_off[c] = o;
    }
    // the pass's gates as (geometry, matrix): as listed, or fused
    std::vector<Geom> pg;
    std::vector<const qcw_c64 *> pu;
    std::vector<qcw_gate> fgates;
    std::vector<qcw_c64> fmats;
    if (fuse) {
      int rc = fuse_gate_list(gates, runs[r].g.data(), (int)runs[r].g.size(), mats, 3,
                              kFuseExtraFlops, (plan & QCW_PLAN_COMMUTE) != 0, &fgates, &fmats);
      if (rc) return rc;
      pg.resize(fgates.size());
      for (size_t i = 0; i < fgates.size(); ++i) {
        if ((rc = make_geom(nq, fgates[i].k, fgates[i].q, &pg[i]))) return rc;
        pu.push_back(fmats.data() + fgates[i].mat);
      }
    } else {
      for (int g : runs[r].g) {
        pg.push_back(geo[g]);
        pu.push_back(mats + gates[g].mat);
      }
    }
    P.ngates = (int)pg.size();
    for (size_t i = 0; i < pg.size(); ++i) {
      const Geom &gg = pg[i];
      FusedGate G;
      memset(&G, 0, sizeof G);
      G.k = gg.k;
      int lb[3] = {0, 0, 0};
      for (int j = 0; j < G.k; ++j) lb[j] = local_of[gg.bit[j]];
      int sl[3] = {lb[0], lb[1], lb[2]};
      std::sort(sl, sl + G.k);
      G.sb0 = sl[0];
      G.sb1 = sl[1];
      G.sb2 = sl[2];
      for (int rr = 0; rr < (1 << G.k); ++rr) {
        uint32_t o = 0;
        for (int j = 0; j < G.k; ++j)
          if ((rr >> (G.k - 1 - j)) & 1) o |= 1u << lb[j];
        G.off[rr] = o;
      }
      const qcw_c64 *U = pu[i];
      G.m3 = (plan & QCW_PLAN_3M) ? 1 : 0;
      for (int e = 0; e < (1 << (2 * G.k)); ++e) {
        if (G.m3) {
          G.u[e] = make_double2(U[e].re, -(U[e].re + U[e].im));
          G.d[e] = U[e].im - U[e].re;
        } else {
          G.u[e] = make_double2(U[e].re, U[e].im);
        }
      }
      fg.push_back(G);
    }
    passes.push_back(P);
  }
  return QCW_OK;
}

// Per-stream device buffer for plans; a stream's previous plan is overwritten
// only by work ordered after that stream's earlier kernels.  The buffer keeps
// the request it was planned for (sig): the same request again reuses the
// plan on the device, with no planning, upload or stream synchronisation.
namespace {
struct PlanBuf {
  void *dev = nullptr;
  size_t bytes = 0;
  std::vector<char> sig;  // request of the plan in dev (empty: none)
  size_t pbytes = 0;      // pass table bytes (the gate table follows)
  int npass = 0;
};
std::mutex g_plan_mu;
std::unordered_map<hipStream_t, PlanBuf> g_plan_bufs;
}  // namespace

// Resident blocks of a pass kernel over the whole device (blocks per CU times
// CUs), for the persistent kernels' grids.  Computed once per (kernel,
// device) under a lock: calls may come from several threads at once.
static int fused_grid(const void *fn, int threads, size_t lds, unsigned *grid) {
  static std::mutex mu;
  static std::map<std::pair<const void *, int>, unsigned> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find({fn, dev});
  if (it != cache.end()) {
    *grid = it->second;
    return QCW_OK;
  }
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return fail(QCW_EHIP, "LDS of %zu B per block: %s", lds, hipGetErrorString(e));
  }
  int bpc = 0, ncu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, fn, threads, lds) != hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "fused occupancy query failed");
  }
  if (bpc < 1) return fail(QCW_EHIP, "fused kernel with %zu B of LDS does not fit a CU", lds);
  *grid = (unsigned)(bpc * ncu);
  cache[{fn, dev}] = *grid;
  return QCW_OK;
}

template <int T, int L, int NT>
static int launch_passes_t(qcw_c64 *psi, int nq, const FusedPass *dp, const FusedGate *dg,
                           int npass, hipStream_t s) {
  const size_t lds = sizeof(double2) << T;
  const uint64_t ntiles = 1ull << (nq - T);
  // 2^13-amplitude tiles fill a CU's LDS with one block, so they run as
  // persistent pipelined blocks; smaller tiles rely on several resident blocks
  // per CU to overlap loads, LDS work and stores (measured faster for them).
  constexpr bool persistent = T >= 13;
  const void *fn = persistent ? (const void *)fused_persistent_kernel<T, L, NT>
                              : (const void *)fused_pass_kernel<T, L, NT>;
  unsigned grid = 0;
  int rc = fused_grid(fn, NT, lds, &grid);
  if (rc) return rc;
  for (int p = 0; p < npass; ++p) {
    TimedLaunch t(QCW_KERNEL_FUSED, s);
    if (persistent) {
      const unsigned blocks = (unsigned)std::min<uint64_t>(grid, ntiles);
      hipLaunchKernelGGL((fused_persistent_kernel<T, L, NT>), dim3(blocks), dim3(NT), lds, s,
                         reinterpret_cast<double2 *>(psi), dp, dg, p, ntiles);
    } else {
      hipLaunchKernelGGL((fused_pass_kernel<T, L, NT>), dim3((unsigned)ntiles), dim3(NT), lds, s,
                         reinterpret_cast<double2 *>(psi), dp, dg, p);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QCW_EHIP, "fused launch: %s", hipGetErrorString(e));
  }
  return QCW_OK;
}

template <int T, int NT>
static int launch_passes_l(int L, qcw_c64 *psi, int nq, const FusedPass *dp, const FusedGate *dg,
                           int np, hipStream_t s) {
  switch (L) {
    case 3: return launch_passes_t<T, 3, NT>(psi, nq, dp, dg, np, s);
    case 4: return launch_passes_t<T, 4, NT>(psi, nq, dp, dg, np, s);
    default: return launch_passes_t<T, 5, NT>(psi, nq, dp, dg, np, s);
  }
}

template <int L>
static int launch_ws(qcw_c64 *psi, int nq, const FusedPass *dp, const FusedGate *dg, int npass,
                     hipStream_t s) {
  constexpr int T = 12;
  const size_t lds = 2 * (sizeof(double2) << T);
  const uint64_t ntiles = 1ull << (nq - T);
  unsigned grid = 0;
  int rc = fused_grid((const void *)fused_ws_kernel<L>, 1024, lds, &grid);
  if (rc) return rc;
  const unsigned blocks = (unsigned)std::min<uint64_t>(grid, ntiles);
  for (int p = 0; p < npass; ++p) {
    TimedLaunch t(QCW_KERNEL_FUSED, s);
    hipLaunchKernelGGL((fused_ws_kernel<L>), dim3(blocks), dim3(1024), lds, s,
                       reinterpret_cast<double2 *>(psi), dp, dg, p, ntiles);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(QCW_EHIP, "fused launch: %s", hipGetErrorString(e));
  }
  return QCW_OK;
}

// Block size per tile size: 256 threads below 2^12 amplitudes; for 2^12 and
// 2^13, 256 / 512 / 1024 threads (threads = 0 picks the tuned default); for
// 2^12, threads = 1024 is the warp-specialised pipelined kernel.
template <int T>
static int launch_passes_n(int threads, int L, qcw_c64 *psi, int nq, const FusedPass *dp,
                           const FusedGate *dg, int np, hipStream_t s) {
  if (threads == 0) threads = fused_block(T);
  if (T == 12 && threads == 1024) {
    switch (L) {
      case 3: return launch_ws<3>(psi, nq, dp, dg, np, s);
      case 4: return launch_ws<4>(psi, nq, dp, dg, np, s);
      default: return launch_ws<5>(psi, nq, dp, dg, np, s);
    }
  }
  switch (threads) {
    case 1024: return launch_passes_l<T, 1024>(L, psi, nq, dp, dg, np, s);
    case 512: return launch_passes_l<T, 512>(L, psi, nq, dp, dg, np, s);
    default: return launch_passes_l<T, 256>(L, psi, nq, dp, dg, np, s);
  }
}

// Uploads a plan into the stream's plan buffer.
static int upload_plan(const std::vector<FusedPass> &passes, const std::vector<FusedGate> &fg,
                       hipStream_t s, std::vector<char> &&sig, const FusedPass **dp,
                       const FusedGate **dg) {
  const size_t pbytes = passes.size() * sizeof(FusedPass);
  const size_t need = pbytes + fg.size() * sizeof(FusedGate);
  void *dev = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    PlanBuf &b = g_plan_bufs[s];
    b.sig.clear();  // until the new plan has landed
    if (b.bytes < need) {
      if (b.dev) {
        // the old buffer may still be read by queued kernels of this stream
        if (hipStreamSynchronize(s) != hipSuccess) return fail(QCW_EHIP, "plan buffer sync");
        (void)hipFree(b.dev);
        b.dev = nullptr;
      }
      size_t nb = std::max<size_t>(need, 1 << 20);
      if (hipMalloc(&b.dev, nb) != hipSuccess) {
        (void)hipGetLastError();
        b.bytes = 0;
        return fail(QCW_ENOMEM, "fused plan buffer (%zu B)", nb);
      }
      b.bytes = nb;
    }
    dev = b.dev;
  }
  std::vector<char> blob(need);
  memcpy(blob.data(), passes.data(), pbytes);
  memcpy(blob.data() + pbytes, fg.data(), fg.size() * sizeof(FusedGate));
  if (hipMemcpyAsync(dev, blob.data(), need, hipMemcpyHostToDevice, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "fused plan upload");
  }
  // the host blob must outlive the (possibly staged) copy
  if (hipStreamSynchronize(s) != hipSuccess) return fail(QCW_EHIP, "fused plan upload sync");
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    PlanBuf &b = g_plan_bufs[s];
    b.sig = std::move(sig);
    b.pbytes = pbytes;
    b.npass = (int)passes.size();
  }
  *dp = (const FusedPass *)dev;
  *dg = (const FusedGate *)((char *)dev + pbytes);
  return QCW_OK;
}

// The request a plan depends on: shape, flags, and every gate's targets and
// matrix entries.
static std::vector<char> plan_signature(int nq, int T, int L, int plan, const qcw_gate *gates,
                                        int ngates, const qcw_c64 *mats) {
  std::vector<char> sig;
  auto put = [&](const void *p, size_t n) {
    const char *c = (const char *)p;
    sig.insert(sig.end(), c, c + n);
  };
  const int head[5] = {nq, T, L, plan, ngates};
  put(head, sizeof head);
  for (int i = 0; i < ngates; ++i) {
    const qcw_gate &g = gates[i];
    put(&g.k, sizeof g.k);
    put(g.q, sizeof(int) * g.k);
    put(mats + g.mat, sizeof(qcw_c64) << (2 * g.k));
  }
  return sig;
}

// ------------------------------------------------------------ no-allocation tables
// qcw_circuit_fused_noalloc keeps its pass and gate tables in this file-scope
// device array instead of a buffer allocated per stream: one copy per GPU,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not a device address; the array's address on each GPU comes from
// hipGetSymbolAddress (scratch_state), and only that address is handed to
// copies and kernels.  Every call on a GPU shares its copy: each call writes
// the whole region its kernels read (nothing needs to start at zero), and
// calls that overlap on one GPU race.
constexpr size_t kScratchBytes = 4u << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
struct ScratchState {
  void *ptr = nullptr;    // device address of `scratch` on this GPU
  std::vector<char> sig;  // request whose plan the array holds (empty: none)
  size_t pbytes = 0;
  int npass = 0;
};
std::mutex g_scratch_mu;
std::map<int, ScratchState> g_scratch;  // per device
}  // namespace

// The current GPU's scratch state; its address is looked up on the first call
// on that GPU (with it current).  The caller holds g_scratch_mu.
static int scratch_state(ScratchState **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return fail(QCW_EHIP, "cannot query the device");
  }
  ScratchState &st = g_scratch[dev];
  if (!st.ptr) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(QCW_EHIP, "device address of the no-allocation buffer: %s", hipGetErrorString(e));
    }
    st.ptr = p;
  }
  *out = &st;
  return QCW_OK;
}

// Places a plan in the current GPU's scratch array (no allocation): reuses it
// when the array already holds this request's plan, else plans, checks the
// size and uploads it on stream s (synchronising s, as upload_plan does).
static int place_plan_in_scratch(int nq, const std::vector<Geom> &geo, const qcw_gate *gates,
                                 const qcw_c64 *mats, FusedShape sh, int plan,
                                 std::vector<char> &&sig, hipStream_t s, const FusedPass **dp,
                                 const FusedGate **dg, int *np) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  ScratchState *st = nullptr;
  int rc = scratch_state(&st);
  if (rc) return rc;
  if (st->sig.empty() || st->sig != sig) {
    std::vector<FusedPass> passes;
    std::vector<FusedGate> fg;
    if ((rc = plan_passes(nq, geo, gates, mats, sh, plan, passes, fg))) return rc;
    const size_t pbytes = passes.size() * sizeof(FusedPass);
    const size_t need = pbytes + fg.size() * sizeof(FusedGate);
    if (need > kScratchBytes)
      return fail(QCW_EINVAL,
                  "the plan's tables (%zu passes, %zu gates: %zu B) exceed the %zu B "
                  "no-allocation buffer; use qcw_circuit_fused_ex",
                  passes.size(), fg.size(), need, kScratchBytes);
    st->sig.clear();  // until the new plan has landed
    std::vector<char> blob(need);
    memcpy(blob.data(), passes.data(), pbytes);
    memcpy(blob.data() + pbytes, fg.data(), fg.size() * sizeof(FusedGate));
    if (hipMemcpyAsync(st->ptr, blob.data(), need, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      (void)hipGetLastError();
      return fail(QCW_EHIP, "upload of the plan into the no-allocation buffer");
    }
    st->sig = std::move(sig);
    st->pbytes = pbytes;
    st->npass = (int)passes.size();
  }
  *dp = (const FusedPass *)st->ptr;
  *dg = (const FusedGate *)((char *)st->ptr + st->pbytes);
  *np = st->npass;
  return QCW_OK;
}

int run_fused(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
              int tile_bits, int low_bits, int threads, int plan, hipStream_t s,
              bool in_scratch) {
  std::vector<Geom> geo(ngates);
  for (int i = 0; i < ngates; ++i) {
    int rc = make_geom(nq, gates[i].k, gates[i].q, &geo[i]);
    if (rc) return rc;
  }
  if (ngates == 0) return QCW_OK;
  // Small states: the whole state is one tile; use the one-gate sweep when a
  // tile would not reach a full block of work.
  const int T = std::min(tile_bits, nq);
  const int L = low_bits;
  if (T < 8 || nq < 9) {
    for (int i = 0; i < ngates; ++i) {
      int rc = launch_sweep(geo[i], mats + gates[i].mat, psi, psi, s);
      if (rc) return rc;
    }
    return QCW_OK;
  }
  const FusedPass *dp = nullptr;
  const FusedGate *dg = nullptr;
  int np = 0;
  std::vector<char> sig = plan_signature(nq, T, L, plan, gates, ngates, mats);
  if (in_scratch) {
    int rc = place_plan_in_scratch(nq, geo, gates, mats, FusedShape{T, L}, plan, std::move(sig),
                                   s, &dp, &dg, &np);
    if (rc) return rc;
  } else {
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      PlanBuf &b = g_plan_bufs[s];
      if (!b.sig.empty() && b.sig == sig) {
        dp = (const FusedPass *)b.dev;
        dg = (const FusedGate *)((char *)b.dev + b.pbytes);
        np = b.npass;
      }
    }
    if (!dp) {
      std::vector<FusedPass> passes;
      std::vector<FusedGate> fg;
      int rc = plan_passes(nq, geo, gates, mats, FusedShape{T, L}, plan, passes, fg);
      if (rc) return rc;
      if ((rc = upload_plan(passes, fg, s, std::move(sig), &dp, &dg))) return rc;
      np = (int)passes.size();
    }
  }
  switch (T) {
    case 8: return launch_passes_l<8, 256>(L, psi, nq, dp, dg, np, s);
    case 9: return launch_passes_l<9, 256>(L, psi, nq, dp, dg, np, s);
    case 10: return launch_passes_l<10, 256>(L, psi, nq, dp, dg, np, s);
    case 11:
      if (threads == 512) return launch_passes_l<11, 512>(L, psi, nq, dp, dg, np, s);
      return launch_passes_l<11, 256>(L, psi, nq, dp, dg, np, s);
    case 12: return launch_passes_n<12>(threads, L, psi, nq, dp, dg, np, s);
    default: return launch_passes_n<13>(threads, L, psi, nq, dp, dg, np, s);
  }
}

int fused_pass_count(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits,
                     int plan, int *pass_of, int *order) {
  std::vector<Geom> geo(ngates);
  for (int i = 0; i < ngates; ++i)
    if (make_geom(nq, gates[i].k, gates[i].q, &geo[i])) return -1;
  const int T = std::min(tile_bits, nq);
  if (T < 8 || nq < 9) {  // one sweep per gate, in list order
    for (int i = 0; i < ngates; ++i) {
      if (pass_of) pass_of[i] = i;
      if (order) order[i] = i;
    }
    return ngates;
  }
  const std::vector<PlanRun> runs =
      plan_runs(nq, geo, FusedShape{T, low_bits}, (plan & QCW_PLAN_COMMUTE) != 0);
  int pos = 0;
  for (size_t r = 0; r < runs.size(); ++r)
    for (int g : runs[r].g) {
      if (pass_of) pass_of[g] = (int)r;
      if (order) order[pos] = g;
      ++pos;
    }
  return (int)runs.size();
}

}  // namespace qcw

using namespace qcw;

extern "C" {

static int fused_entry(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                       const qcw_c64 *mats, int64_t nmats, int tile_bits, int low_bits,
                       int threads, int plan, void *stream, bool in_scratch) {
  clear_error();
  if (plan & ~(QCW_PLAN_COMMUTE | QCW_PLAN_FUSE | QCW_PLAN_3M))
    return fail(QCW_EINVAL, "plan=%d has bits other than QCW_PLAN_COMMUTE, QCW_PLAN_FUSE and QCW_PLAN_3M", plan);
  if (nq < 1 || nq > kMaxQubits) return fail(QCW_EINVAL, "nq=%d outside [1, %d]", nq, kMaxQubits);
  if (ngates < 0) return fail(QCW_EINVAL, "ngates < 0");
  if (ngates > 0 && (!gates || !mats)) return fail(QCW_EINVAL, "gates or mats is NULL");
  if (tile_bits == 0) tile_bits = kFusedDefaultTile;
  if (low_bits == 0) low_bits = kFusedDefaultLow;
  if (tile_bits < 8 || tile_bits > 13) return fail(QCW_EINVAL, "tile_bits=%d outside [8, 13]", tile_bits);
  if (low_bits < 3 || low_bits > 5 || tile_bits - low_bits > kFusedMaxFree)
    return fail(QCW_EINVAL, "low_bits=%d outside [3, 5] or too few for tile_bits=%d", low_bits, tile_bits);
  if (threads != 0 && !((threads == 256 || threads == 512 || threads == 1024) && tile_bits >= 12) &&
      !((threads == 256 || threads == 512) && tile_bits == 11))
    return fail(QCW_EINVAL, "threads=%d: 256/512 (tile_bits 11), 256/512/1024 (12, 13), or 0", threads);
  for (int i = 0; i < ngates; ++i) {
    Geom g;
    int rc = make_geom(nq, gates[i].k, gates[i].q, &g);
    if (rc) {
      char why[400];
      snprintf(why, sizeof why, "%s", last_error());
      return fail(rc, "gate %d: %s", i, why);
    }
    const int64_t mm = (int64_t)1 << (2 * gates[i].k);
    if (gates[i].mat < 0 || gates[i].mat + mm > nmats)
      return fail(QCW_EINVAL, "gate %d: matrix offset outside mats", i);
  }
  int rc = check_device_range(psi, ((uint64_t)1 << nq) * sizeof(qcw_c64), "psi");
  if (rc) return rc;
  return run_fused(psi, nq, gates, ngates, mats, tile_bits, low_bits, threads, plan,
                   (hipStream_t)stream, in_scratch);
}

int qcw_circuit_fused_ex(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                         const qcw_c64 *mats, int64_t nmats, int tile_bits, int low_bits,
                         int threads, int plan, void *stream) {
  return fused_entry(psi, nq, gates, ngates, mats, nmats, tile_bits, low_bits, threads, plan,
                     stream, false);
}

int qcw_circuit_fused_noalloc(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                              const qcw_c64 *mats, int64_t nmats, int tile_bits, int low_bits,
                              int threads, int plan, void *stream) {
  return fused_entry(psi, nq, gates, ngates, mats, nmats, tile_bits, low_bits, threads, plan,
                     stream, true);
}

int qcw_circuit_fused(qcw_c64 *psi, int nq, const qcw_gate *gates, int ngates,
                      const qcw_c64 *mats, int64_t nmats, int tile_bits, void *stream) {
  return qcw_circuit_fused_ex(psi, nq, gates, ngates, mats, nmats, tile_bits, 0, 0, 0, stream);
}

int qcw_fused_pass_count(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits,
                         int plan) {
  clear_error();
  if (tile_bits == 0) tile_bits = kFusedDefaultTile;
  if (low_bits == 0) low_bits = kFusedDefaultLow;
  if (nq < 1 || nq > kMaxQubits || ngates < 0 || (ngates > 0 && !gates) || tile_bits < 8 ||
      tile_bits > 13 || low_bits < 3 || low_bits > 5 || tile_bits - low_bits > kFusedMaxFree ||
      (plan & ~(QCW_PLAN_COMMUTE | QCW_PLAN_FUSE | QCW_PLAN_3M)))
    return fail(QCW_EINVAL, "invalid arguments");
  int n = fused_pass_count(nq, gates, ngates, tile_bits, low_bits, plan, nullptr, nullptr);
  return n < 0 ? fail(QCW_EINVAL, "invalid gate") : n;
}

int qcw_fused_plan(int nq, const qcw_gate *gates, int ngates, int tile_bits, int low_bits,
                   int plan, int *pass_of, int *order) {
  clear_error();
  if (tile_bits == 0) tile_bits = kFusedDefaultTile;
  if (low_bits == 0) low_bits = kFusedDefaultLow;
  if (nq < 1 || nq > kMaxQubits || ngates < 0 || (ngates > 0 && (!gates || !pass_of || !order)) ||
      tile_bits < 8 || tile_bits > 13 || low_bits < 3 || low_bits > 5 ||
      tile_bits - low_bits > kFusedMaxFree || (plan & ~(QCW_PLAN_COMMUTE | QCW_PLAN_FUSE | QCW_PLAN_3M)))
    return fail(QCW_EINVAL, "invalid arguments");
  int n = fused_pass_count(nq, gates, ngates, tile_bits, low_bits, plan, pass_of, order);
  return n < 0 ? fail(QCW_EINVAL, "invalid gate") : n;
}


int qcw_debug_fused_tables(int nq, const qcw_gate *gates, int ngates, const qcw_c64 *mats,
                           int64_t nmats, int tile_bits, int low_bits, int plan, int pass_cap,
                           int gate_cap, int32_t *pass_hdr, int32_t *outer_pos,
                           uint64_t *chunk_off, int32_t *gate_hdr, qcw_c64 *gate_mat,
                           int *npass, int *ngate) {
  clear_error();
  if (tile_bits == 0) tile_bits = kFusedDefaultTile;
  if (low_bits == 0) low_bits = kFusedDefaultLow;
  if (nq < 9 || nq > kMaxQubits || ngates < 1 || !gates || !mats || tile_bits < 8 ||
      tile_bits > 13 || low_bits < 3 || low_bits > 5 || tile_bits - low_bits > kFusedMaxFree ||
      (plan & ~(QCW_PLAN_COMMUTE | QCW_PLAN_FUSE | QCW_PLAN_3M)) || !pass_hdr || !outer_pos ||
      !chunk_off || !gate_hdr || !gate_mat || !npass || !ngate)
    return fail(QCW_EINVAL, "invalid arguments");
  std::vector<Geom> geo(ngates);
  for (int i = 0; i < ngates; ++i) {
    int rc = make_geom(nq, gates[i].k, gates[i].q, &geo[i]);
    if (rc) return rc;
    const int64_t mm = (int64_t)1 << (2 * gates[i].k);
    if (gates[i].mat < 0 || gates[i].mat + mm > nmats)
      return fail(QCW_EINVAL, "gate %d: matrix offset outside mats", i);
  }
  std::vector<FusedPass> passes;
  std::vector<FusedGate> fg;
  int rc = plan_passes(nq, geo, gates, mats, FusedShape{std::min(tile_bits, nq), low_bits}, plan,
                       passes, fg);
  if (rc) return rc;
  *npass = (int)passes.size();
  *ngate = (int)fg.size();
  if ((int)passes.size() > pass_cap || (int)fg.size() > gate_cap)
    return fail(QCW_EINVAL, "plan has %zu passes and %zu gates (caps %d, %d)", passes.size(),
                fg.size(), pass_cap, gate_cap);
  for (size_t p = 0; p < passes.size(); ++p) {
    const FusedPass &P = passes[p];
    pass_hdr[4 * p + 0] = P.gate_off;
    pass_hdr[4 * p + 1] = P.ngates;
    pass_hdr[4 * p + 2] = P.T;
    pass_hdr[4 * p + 3] = P.L;
    for (int j = 0; j < 40; ++j) outer_pos[40 * p + j] = j < P.n_outer ? P.outer_pos[j] : -1;
    for (int c = 0; c < (1 << kFusedMaxFree); ++c) chunk_off[(1 << kFusedMaxFree) * p + c] = P.chunk_off[c];
  }
  for (size_t g = 0; g < fg.size(); ++g) {
    const FusedGate &G = fg[g];
    int32_t *h = gate_hdr + 13 * g;
    h[0] = G.k;
    h[1] = G.sb0;
    h[2] = G.sb1;
    h[3] = G.sb2;
    h[4] = G.m3;
    for (int r = 0; r < 8; ++r) h[5 + r] = (int32_t)G.off[r];
    for (int e = 0; e < 64; ++e) gate_mat[64 * g + e] = qcw_c64{G.u[e].x, G.u[e].y};
  }
  return QCW_OK;
}

}  // extern "C"

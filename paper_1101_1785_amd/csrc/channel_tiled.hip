// Tiled form of the multiverse channel (QCWAVE §5, Eqs. rhoE1 and rhoE4) for
// channels whose path operators are products of permutation-type one-qubit
// operators (Pauli operators, phases, the identity).
//
// A permutation-type term links output (n, m) with input (n ^ f, m ^ f) for
// its flip mask f, times a coefficient that depends only on the bits of n
// and m at the term's qubits.  Terms with the same f form a group: one read
// of rho per output, one combined coefficient, tabulated on the host over
// the bits (n_b, m_b) of the group's qubits (in segments of at most three
// qubits, each segment's table the sum of its terms' coefficient products).
//
// Tile.  For two bits E0 < E1 chosen on the host from bits 4 .. nq-1 and a
// tile base (nb, mb) whose bits 0..3 are zero (and, in nb, bits E0 and E1),
// the tile holds the 1024 elements
//     n = nb | dep(a) | r,   m = (mb ^ dep(a)) | c,     a < 4, r, c < 16,
// where dep(a) puts bit 0 of a at E0 and bit 1 at E1.  A flip f, split into
// f_lo (bits 0..3), f_E (its bits at E0, E1, as a 2-bit number) and f_R (the
// rest), maps element (a, r, c) of this tile to element
// (a ^ f_E, r ^ f_lo, c ^ f_lo) of the tile at (nb ^ f_R, mb ^ f_R).  A
// workgroup owning a tile therefore reads rho only on its partner tiles, one
// per distinct f_R among the channel's flips (f_R = 0: the tile itself).
// Thread (r, c) owns the four outputs a < 4 at its (r, c).  For a partner
// and a value of f_lo (a read set) it reads the four partner elements at
// (b, r ^ f_lo, c ^ f_lo), b < 4, once, and every group of that read set
// uses them, output a taking element a ^ f_E.  A partner read by two or more
// read sets is staged in LDS (coalesced loads, then LDS reads); one read by a
// single read set is read from memory directly.  A group whose qubits avoid
// E0 and E1 has one coefficient for all four outputs of a thread.
//
// Tiles with the same n ^ m above bit 3 (a family of 2^(nq-6) tiles) are
// closed under every flip.  Workgroups are dealt to the 8 XCDs in turn and
// each XCD works through its own families, so partner reads stay in that
// XCD's L2.
#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "channel_tiled.h"
#include "qcw_common.h"
#include "rtc.h"

#include "qcw.h"

namespace qcw {

namespace {

constexpr int kTileThreads = 256;             // thread (r, c), r, c < 16
constexpr int kTileElems = 1024;              // four elements per thread
constexpr int kRound = 2;                     // partners whose loads are issued together
constexpr int kSegMaxQubits = 3;              // a segment's table has at most 64 entries
constexpr uint32_t kZeroField = 30;           // bits 30..31 of the interleaved index: zero
constexpr size_t kTableBytesMax = 32 << 10;   // coefficient tables staged in LDS

enum PartnerMode : int32_t { kOwn = 0, kStaged = 1, kDirect = 2 };

constexpr uint32_t kTicketSubs = 8;     // ticket counters per XCD, at most
constexpr uint32_t kTicketStride = 32;  // words between counters: one 128-byte line each

// One segment: its table entry for an output with interleaved index nm is
// entry f0 + 4 f1 + 16 f2 of its table (4^k entries for k qubits), f_j =
// (nm >> sh_j) & 3 for its j-th qubit (for qubit bit b, (nm >> 2b) & 3 =
// (n_b << 1) | m_b).  A segment of fewer than three qubits reads its missing
// fields at bits 30..31 of nm, zero for nq <= 15.  The first record of a
// group is its first segment; `extra` records follow.
struct TRec {
  uint32_t sh0, sh1, sh2;
  uint32_t entry_b;  // LDS byte address of its table
  uint32_t etouch;   // a qubit is E0 or E1: the four outputs of a thread differ
  uint32_t extra;    // (first record of a group) further segments of the group
  uint32_t nbits;    // qubits of the segment, 1..3
  uint32_t pad;
};
// Kinds of groups in a read set, in stream order: for f_E = 0..3, the groups
// with one coefficient for the thread's four outputs, then the others (whose
// first segment is one on E0 or E1).
constexpr int kKinds = 8;
struct TRead {
  uint32_t flo17;           // f_lo * 17: the flip of the thread index r * 16 + c
  uint32_t rec;             // first record
  uint32_t count[kKinds];   // groups of each kind
  uint32_t kinds;           // bit k set: count[k] > 0
  uint32_t pad;
};
struct TPartner {
  uint64_t fRb;   // byte flip of the tile base: ((f_R << nq) | f_R) * 16
  int32_t mode;
  uint32_t r_first, r_count;
  uint32_t lflob; // byte flip of the thread's loads: ((f << nq) | f) * 16 for f = f_lo when
                  // the partner is read directly, 0 when staged
  uint32_t pad[2];
};

struct TArgs {
  int nq, e0, e1, mb_bits;  // mb_bits: log2 of the tiles of a family
  double p_keep;
  uint32_t xcd_tiles;       // tiles each XCD works through (all tiles / 8)
  uint32_t xcd_blocks;      // blocks on each XCD (grid / 8)
  uint32_t nsub;            // ticket counters per XCD (each XCD has at least nsub blocks)
  uint32_t *tickets;        // per XCD x: counters x * kTicketSubs + s; blocks finished 8 * kTicketSubs + x
                            // (each in its own kTicketStride words)
  int npartners;
  int own_staged, any_staged;
  int tab_entries;
  const TPartner *partners;
  const TRead *reads;
  const TRec *recs;
  const void *tables;
};

template <bool REAL>
struct CoefT;
template <>
struct CoefT<true> {
  using T = double;
};
template <>
struct CoefT<false> {
  using T = double2;
};

__device__ __forceinline__ void cacc(double &a, double b) { a += b; }
__device__ __forceinline__ void cacc(double2 &a, double2 b) {
  a.x += b.x;
  a.y += b.y;
}
__device__ __forceinline__ void madd(double2 &acc, double c, double2 v) {
  acc.x = __fma_rn(c, v.x, acc.x);
  acc.y = __fma_rn(c, v.y, acc.y);
}
__device__ __forceinline__ void madd(double2 &acc, double2 c, double2 v) {
  acc.x = __fma_rn(c.x, v.x, acc.x);
  acc.x = __fma_rn(-c.y, v.y, acc.x);
  acc.y = __fma_rn(c.x, v.y, acc.y);
  acc.y = __fma_rn(c.y, v.x, acc.y);
}

// Descriptor reads through the constant address space: the plan is never
// written by the kernel, and as generic pointers the compiler would read it
// with vector loads (it cannot rule out aliasing with the output stores),
// whose waits also drain the partner loads in flight.  The byte offset is
// wave-uniform; readfirstlane keeps it in a scalar register.  (Word by word:
// a struct cannot be copied out of that address space.)
template <typename T>
__device__ __forceinline__ T ldc(const void *base, uint32_t off) {
  static_assert(sizeof(T) % 4 == 0, "descriptor of whole words");
  off = __builtin_amdgcn_readfirstlane(off);
  const __attribute__((address_space(4))) uint32_t *w =
      (const __attribute__((address_space(4))) uint32_t *)((const char *)base + off);
  T r;
  uint32_t *o = reinterpret_cast<uint32_t *>(&r);
#pragma unroll
  for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = w[k];
  return r;
}

template <typename CT>
__device__ __forceinline__ CT entry_at(const TRec &S, uint32_t nm, const char *lds) {
  const uint32_t i = __builtin_amdgcn_ubfe(nm, S.sh0, 2) | (__builtin_amdgcn_ubfe(nm, S.sh1, 2) << 2) |
                     (__builtin_amdgcn_ubfe(nm, S.sh2, 2) << 4);
  return *reinterpret_cast<const CT *>(lds + S.entry_b + i * sizeof(CT));
}

// The groups of one kind: f_E = FE; UNI: every segment avoids E0 and E1, so
// one coefficient serves the thread's four outputs.  acc[a] += c[a] v[a ^ FE].
// Returns the record after the last one read.
template <int FE, bool UNI, bool REAL>
__device__ __forceinline__ uint32_t run_kind(double2 (&acc)[4], const double2 (&v)[4], const TRec *recs,
                                             uint32_t ob, uint32_t n, uint32_t nm0,
                                             const uint32_t (&K)[4], const char *lds) {
  using CT = typename CoefT<REAL>::T;
  for (uint32_t g = 0; g < n; ++g) {
    const TRec G = ldc<TRec>(recs, ob);
    ob += sizeof(TRec);
    if (UNI) {
      CT c = entry_at<CT>(G, nm0, lds);
      for (uint32_t e = 0; e < G.extra; ++e, ob += sizeof(TRec)) cacc(c, entry_at<CT>(ldc<TRec>(recs, ob), nm0, lds));
#pragma unroll
      for (int a = 0; a < 4; ++a) madd(acc[a], c, v[a ^ FE]);
    } else {
      CT c[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) c[a] = entry_at<CT>(G, nm0 ^ K[a], lds);  // first segment: on E0/E1
      for (uint32_t e = 0; e < G.extra; ++e, ob += sizeof(TRec)) {
        const TRec S = ldc<TRec>(recs, ob);
        if (S.etouch) {
#pragma unroll
          for (int a = 0; a < 4; ++a) cacc(c[a], entry_at<CT>(S, nm0 ^ K[a], lds));
        } else {
          const CT t = entry_at<CT>(S, nm0, lds);
#pragma unroll
          for (int a = 0; a < 4; ++a) cacc(c[a], t);
        }
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) madd(acc[a], c[a], v[a ^ FE]);
    }
  }
  return ob;
}

template <bool REAL>
__device__ __forceinline__ void run_read(double2 (&acc)[4], const double2 (&v)[4], const TRead &R,
                                         const TArgs &A, uint32_t nm0, const uint32_t (&K)[4],
                                         const char *lds) {
  uint32_t ob = R.rec * (uint32_t)sizeof(TRec);
  ob = run_kind<0, true, REAL>(acc, v, A.recs, ob, R.count[0], nm0, K, lds);
  ob = run_kind<0, false, REAL>(acc, v, A.recs, ob, R.count[1], nm0, K, lds);
  ob = run_kind<1, true, REAL>(acc, v, A.recs, ob, R.count[2], nm0, K, lds);
  ob = run_kind<1, false, REAL>(acc, v, A.recs, ob, R.count[3], nm0, K, lds);
  ob = run_kind<2, true, REAL>(acc, v, A.recs, ob, R.count[4], nm0, K, lds);
  ob = run_kind<2, false, REAL>(acc, v, A.recs, ob, R.count[5], nm0, K, lds);
  ob = run_kind<3, true, REAL>(acc, v, A.recs, ob, R.count[6], nm0, K, lds);
  (void)run_kind<3, false, REAL>(acc, v, A.recs, ob, R.count[7], nm0, K, lds);
}

typedef double dbl2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ size_t el(uint32_t n, uint32_t m, int nq) {
  return ((size_t)n << nq) | m;
}

// out = p rho + sum over groups of c(n, m) rho(n ^ f, m ^ f), one tile per
// workgroup iteration (persistent: blocks stride over the tiles).
template <bool REAL>
__global__ __launch_bounds__(kTileThreads) void channel_tiled_kernel(const double2 *__restrict__ rho,
                                                                     double2 *__restrict__ out,
                                                                     TArgs A) {
  using CT = typename CoefT<REAL>::T;
  extern __shared__ double2 lds[];
  double2 *own_slot = lds;
  double2 *part_slot = lds + (A.own_staged ? kTileElems : 0);
  CT *tab = reinterpret_cast<CT *>(part_slot + (A.any_staged ? kTileElems : 0));
  {
    const CT *g = static_cast<const CT *>(A.tables);
    for (int i = threadIdx.x; i < A.tab_entries; i += kTileThreads) tab[i] = g[i];
  }
  const int nq = A.nq;
  const uint32_t tid = threadIdx.x, r = tid >> 4, c = tid & 15u;
  const uint32_t d1 = 1u << A.e0, d2 = 1u << A.e1;
  const uint32_t dep[4] = {0u, d1, d2, d1 | d2};
  uint64_t db[4];  // byte offsets of the tile's four blocks from its first
#pragma unroll
  for (int b = 0; b < 4; ++b) db[b] = (((uint64_t)dep[b] << nq) | dep[b]) << 4;
  const uint32_t k1 = 3u << (2 * A.e0), k2 = 3u << (2 * A.e1);
  const uint32_t K[4] = {0u, k1, k2, k1 | k2};
  const uint32_t mmask = (1u << A.mb_bits) - 1u;
  const uint32_t t0b = ((r << nq) | c) << 4;  // this thread's byte offset within a tile's rows
  // Block b runs on XCD b mod 8.  Each XCD takes its families (family ==
  // XCD mod 8) in order, and its blocks draw the next tile of that sequence
  // from the XCD's ticket counters, so the tiles in flight on an XCD stay a
  // window of consecutive tiles, mostly one family, whose partners share
  // its L2 (a fixed stride would let blocks drift apart over the launch).
  // An XCD has `nsub` counters, each on its own cache line: counter s hands
  // out the tiles j == s mod nsub to its blocks (atomics on one address
  // serialise: one counter for all of an XCD's blocks took as long as moving
  // the tiles).  The next ticket is drawn at the start of the current tile
  // and published at the next tile start, so the atomic's latency overlaps a
  // tile's work.  (The library is built without the compiler's wave-level
  // atomic combining, which would read the drawn value right after the
  // atomic and so wait for its round trip there.)
  const uint32_t x = blockIdx.x & 7u;
  const uint32_t sub = (blockIdx.x >> 3) % A.nsub;
  uint32_t *counter = A.tickets + (x * kTicketSubs + sub) * kTicketStride;
  __shared__ uint32_t s_ticket[2];
  uint32_t drawn = 0;  // the counter's value; its ticket is drawn * nsub + sub
  if (threadIdx.x == 0) drawn = atomicAdd(counter, 1u);
  for (uint32_t it = 0;; ++it) {
    if (threadIdx.x == 0) s_ticket[it & 1u] = drawn * A.nsub + sub;
    // Also the tile-start barrier: the previous tile's LDS reads are done
    // (first time: tables copied).  The ticket slot alternates, so the next
    // one cannot overwrite one still being read.
    __syncthreads();
    const uint32_t j = s_ticket[it & 1u];
    if (j >= A.xcd_tiles) break;
    if (threadIdx.x == 0) drawn = atomicAdd(counter, 1u);
    const uint32_t family = ((j >> A.mb_bits) << 3) | x;
    uint32_t nb = (j & mmask) << 4;  // the member's bits, zeros inserted at E0 and E1
    nb = ((nb >> A.e0) << (A.e0 + 1)) | (nb & (d1 - 1u));
    nb = ((nb >> A.e1) << (A.e1 + 1)) | (nb & (d2 - 1u));
    const uint32_t mb = nb ^ (family << 4);
    const uint32_t n0 = nb | r, m0 = mb | c;
    const uint32_t nm0 = (spread16(n0) << 1) | spread16(m0);
    // Element (b, r', c') of the tile at (nb ^ f, mb ^ f) is at byte
    // U0 ^ F ^ D(b) + (r' << nq | c') * 16, with U0 = (nb << nq | mb) * 16,
    // F = (f << nq | f) * 16 and D(b) = (dep(b) << nq | dep(b)) * 16 (the
    // fields do not overlap, so the flips are XORs): a wave-uniform scalar
    // base and a 32-bit per-thread byte offset.
    const uint64_t u0 = (((uint64_t)nb << nq) | mb) << 4;
    auto at = [&](const double2 *base, uint64_t fb, int b, uint32_t off_b) {
      return *reinterpret_cast<const double2 *>(reinterpret_cast<const char *>(base) +
                                                (u0 ^ fb ^ db[b]) + off_b);
    };
    double2 own[4], acc[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) own[a] = at(rho, 0, a, t0b);
    // Partners 1.. in rounds of kRound: every load of a round is issued before
    // the first of its partners is used, so their latencies overlap (round 1
    // also with the tile's own work).  Slots past the last partner load
    // nothing; only a round that ends early then waits for all of its loads
    // at once.
    double2 q[kRound][4];
    auto issue = [&](int p1) {
#pragma unroll
      for (int k = 0; k < kRound; ++k) {
        if (k > 0 && p1 + k >= A.npartners) break;
        const TPartner P = ldc<TPartner>(A.partners, (uint32_t)(p1 + k) * (uint32_t)sizeof(TPartner));
        const uint32_t off_b = t0b ^ P.lflob;
#pragma unroll
        for (int b = 0; b < 4; ++b) q[k][b] = at(rho, P.fRb, b, off_b);
      }
    };
    if (A.npartners > 1) issue(1);
    if (A.own_staged) {
#pragma unroll
      for (int a = 0; a < 4; ++a) own_slot[a * 256 + tid] = own[a];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) acc[a] = make_double2(0.0, 0.0);
    // One partner's read sets; qk: its loads (direct) or the values to stage.
    auto process = [&](const TPartner &P, const double2 (&qk)[4]) {
      if (P.mode == kStaged) {
        __syncthreads();  // readers of the previous staged partner are done
#pragma unroll
        for (int b = 0; b < 4; ++b) part_slot[b * 256 + tid] = qk[b];
        __syncthreads();
      } else if (P.mode == kOwn && A.own_staged) {
        __syncthreads();  // the own tile is in LDS
      }
      for (uint32_t ri = P.r_first; ri < P.r_first + P.r_count; ++ri) {
        const TRead R = ldc<TRead>(A.reads, ri * (uint32_t)sizeof(TRead));
        double2 v[4];
        if (P.mode == kOwn && R.flo17 == 0) {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[b] = own[b];
        } else if (P.mode == kOwn) {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[b] = own_slot[b * 256 + (tid ^ R.flo17)];
        } else if (P.mode == kStaged) {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[b] = part_slot[b * 256 + (tid ^ R.flo17)];
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b) v[b] = qk[b];
        }
        run_read<REAL>(acc, v, R, A, nm0, K, reinterpret_cast<const char *>(lds));
      }
    };
    process(ldc<TPartner>(A.partners, 0u), own);
    for (int p1 = 1; p1 < A.npartners; p1 += kRound) {
      if (p1 > 1) issue(p1);
#pragma unroll
      for (int k = 0; k < kRound; ++k) {
        const int p = p1 + k;
        if (p >= A.npartners) break;
        process(ldc<TPartner>(A.partners, (uint32_t)p * (uint32_t)sizeof(TPartner)), q[k]);
      }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      acc[a].x = __fma_rn(A.p_keep, own[a].x, acc[a].x);
      acc[a].y = __fma_rn(A.p_keep, own[a].y, acc[a].y);
    }
    // Non-temporal stores: the output is not read again by this launch, and
    // left in L2 it would evict the family's tiles that partners still read.
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const dbl2v w = {acc[a].x, acc[a].y};
      __builtin_nontemporal_store(w, reinterpret_cast<dbl2v *>(reinterpret_cast<char *>(out) +
                                                               (u0 ^ db[a]) + t0b));
    }
  }
  // The last block of the XCD to finish (every block of it has drawn its
  // last ticket) clears the XCD's counters for the next launch.
  uint32_t *done = A.tickets + (8 * kTicketSubs + x) * kTicketStride;
  if (threadIdx.x == 0 && atomicAdd(done, 1u) == A.xcd_blocks - 1u) {
    for (uint32_t k = 0; k < A.nsub; ++k) atomicExch(A.tickets + (x * kTicketSubs + k) * kTicketStride, 0u);
    atomicExch(done, 0u);
  }
}

// Inputs of the source generator (tiled_source, below).
struct GenPlan {
  int nq, e0, e1, mb_bits;
  uint32_t xcd_tiles;
  bool real, own_staged, any_staged;
  size_t tab_entries;
  // Order of the tiles of a family: member = sum over set bits k of the
  // ticket's member field of member_basis[k] (XOR); coset_order false: the
  // member is the field itself.
  bool coset_order;
  uint32_t member_basis[32];
  const std::vector<TPartner> *partners;
  const std::vector<TRead> *reads;
  const std::vector<TRec> *recs;  // entry_b still the table entry index
};

const void *tiled_fn(bool real) {
  return real ? reinterpret_cast<const void *>(&channel_tiled_kernel<true>)
              : reinterpret_cast<const void *>(&channel_tiled_kernel<false>);
}

}  // namespace

struct TiledChannel {
  TArgs args{};
  bool real = false;
  void *dbuf = nullptr;  // descriptors and tables, one allocation
  size_t lds = 0;
  unsigned grid = 0;
  int64_t flops = 0;
  TiledSummary sum{};
  const RtcKernel *spec = nullptr;  // the kernel compiled for this plan
  unsigned spec_grid = 0;
  uint32_t spec_xcd_blocks = 0, spec_nsub = 0;
  // generator inputs, for the kernels with permuted stores
  GenPlan gen{};
  std::vector<TPartner> g_partners;
  std::vector<TRead> g_reads;
  std::vector<TRec> g_recs;
  int ncu = 0;
  struct Launch {
    const RtcKernel *k = nullptr;
    unsigned grid = 0;
    uint32_t xcd_blocks = 0, nsub = 0;
    int obs = 0;         // the kernel takes psi0 and part
    int gate_words = 0;  // doubles of a general gate's matrix argument (0: none)
  };
  mutable std::mutex perm_mu;
  mutable std::map<std::vector<int>, Launch> perm_kernels;  // by gate (k, bits, table)
};

namespace {

// Hits of one group split into segments of at most kSegMaxQubits qubits, in
// input order (a hit joins the first segment it fits).
struct SegBuild {
  std::vector<int> bits;  // ascending
  std::vector<const PermTerm *> hits;
};

std::vector<SegBuild> make_segments(const std::vector<const PermTerm *> &hits) {
  std::vector<SegBuild> segs;
  for (const PermTerm *h : hits) {
    std::vector<int> hb = {h->bit0};
    if (h->nops == 2) hb.push_back(h->bit1);
    bool placed = false;
    for (SegBuild &s : segs) {
      std::set<int> u(s.bits.begin(), s.bits.end());
      u.insert(hb.begin(), hb.end());
      if ((int)u.size() <= kSegMaxQubits) {
        s.bits.assign(u.begin(), u.end());
        s.hits.push_back(h);
        placed = true;
        break;
      }
    }
    if (!placed) {
      SegBuild s;
      s.bits = hb;
      std::sort(s.bits.begin(), s.bits.end());
      s.hits.push_back(h);
      segs.push_back(s);
    }
  }
  return segs;
}

// Table of a segment, 4^k entries for its k qubits: entry f0 + 4 f1 + 16 f2,
// with f_j = (n_b << 1) | m_b of its j-th qubit, is the sum over its hits of
// c0(n_b0, m_b0) [c1(n_b1, m_b1)].
std::vector<double2> segment_table(const SegBuild &s) {
  std::vector<double2> t(1u << (2 * s.bits.size()));
  auto field = [&](uint32_t i, int bit) {
    const int j = (int)(std::find(s.bits.begin(), s.bits.end(), bit) - s.bits.begin());
    return (i >> (2 * j)) & 3u;
  };
  for (uint32_t i = 0; i < t.size(); ++i) {
    double2 sum = make_double2(0.0, 0.0);
    for (const PermTerm *h : s.hits) {
      double2 v = h->c0[field(i, h->bit0)];
      if (h->nops == 2) {
        const double2 w = h->c1[field(i, h->bit1)];
        v = make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
      }
      sum.x += v.x;
      sum.y += v.y;
    }
    t[i] = sum;
  }
  return t;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Ticket counters per XCD for a grid of xcd_blocks blocks per XCD: a power of
// two, at most kTicketSubs, each counter serving at least two blocks.
uint32_t ticket_subs(uint32_t xcd_blocks) {
  uint32_t n = 1;
  while (n < kTicketSubs && 2 * n <= xcd_blocks) n *= 2;
  return n;
}

// ---------------------------------------------------------------------------
// The kernel specialised to one plan, compiled at run time.  It is the tiled
// kernel above with the plan's descriptors turned into code: partner flips,
// read sets, group kinds and segment qubits become constants, so nothing is
// decoded per group.  A segment's table index is split into the fields of
// its qubits at bits 0..3 (fixed per thread for the whole launch: hoisted
// out of the tile loop) and the others (the same for the whole tile, or for
// one output a on E0/E1: scalar arithmetic).  The thread fields are the
// low digits of the index (a segment's qubits are in ascending bit order),
// so the two parts add.  Groups, segments and products run in the generic
// kernel's order with its operations, so the two kernels agree bit for bit.


void add(std::string &s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void add(std::string &s, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  s += buf;
}

constexpr const char *kSpecName = "qcw_channel_tiled_spec";
// Resident blocks per CU for the compiled kernel.  With four, the tiles in
// flight on an XCD (and the partner tiles they read) outgrow its L2 and the
// partner reads go back to memory: at nq = 13 the HBM reads per launch were
// 2.3 times the state, against 1.2 times with three, which also ran faster
// (0.53 ms against 0.55; two: 0.58).  At nq = 12 two ran fastest (0.111 ms,
// three 0.132, four 0.166); at nq = 14 two and three tie.
int spec_blocks_per_cu(int nq) { return nq <= 12 ? 2 : 3; }

// obs: 0 no observables; 1 trace and purity; 2 also the fidelity against
// psi0.  (Two variants rather than a branch on psi0: with the branch the
// compiler's code for the tile loop needed 286 VGPRs instead of 130.)
std::string tiled_source(const GenPlan &G, const OutPerm *gate, int obs) {
  const int nq = G.nq, e0 = G.e0, e1 = G.e1;
  // a monomial gate moves the stores; a general gate on bits 0..3 runs on
  // the tile's outputs in LDS (its matrix arrives with each launch)
  const OutPerm *perm = gate && !gate->general ? gate : nullptr;
  const OutPerm *low = gate && gate->general ? gate : nullptr;
  const int gm = low ? 1 << low->k : 0;
  uint32_t gmask = 0;
  for (int j = 0; low && j < low->k; ++j) gmask |= 1u << low->bits[j];
  const std::vector<TPartner> &P = *G.partners;
  const std::vector<TRead> &R = *G.reads;
  const std::vector<TRec> &S = *G.recs;
  std::string s;
  // the uniform fields the segments need
  std::set<int> ubits;
  bool need_e0 = false, need_e1 = false;
  for (const TRec &rc : S)
    for (uint32_t j = 0; j < rc.nbits; ++j) {
      const int b = (int)((j == 0 ? rc.sh0 : j == 1 ? rc.sh1 : rc.sh2) / 2);
      if (b == e0) need_e0 = true;
      else if (b == e1) need_e1 = true;
      else if (b >= 4) ubits.insert(b);
    }
  add(s, "typedef unsigned int u32;\ntypedef unsigned long long u64;\n");
  add(s, "typedef double dbl2v __attribute__((ext_vector_type(2)));\n");
  add(s, "typedef %s CT;\n", G.real ? "double" : "double2");
  s += R"(
__device__ __forceinline__ void madd(double2 &acc, double c, double2 v) {
  acc.x = __fma_rn(c, v.x, acc.x);
  acc.y = __fma_rn(c, v.y, acc.y);
}
__device__ __forceinline__ void madd(double2 &acc, double2 c, double2 v) {
  acc.x = __fma_rn(c.x, v.x, acc.x);
  acc.x = __fma_rn(-c.y, v.y, acc.x);
  acc.y = __fma_rn(c.x, v.y, acc.y);
  acc.y = __fma_rn(c.y, v.x, acc.y);
}
__device__ __forceinline__ double cadd(double a, double b) { return a + b; }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) {
  a.x += b.x;
  a.y += b.y;
  return a;
}
)";
  if (obs) {
    // A wave's sum of one double with data-parallel-primitive moves: pairs
    // and quads (quad permutations), rows of 16 (half-row and row mirrors),
    // then the row-15 and row-31 broadcasts carry the row totals up, so that
    // lane 63 ends with all 64.  Masked-off rows take the +0 start value.
    s += R"(template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const u64 b = __builtin_bit_cast(u64, v);
  const u32 lo = __builtin_amdgcn_update_dpp(0, (int)(u32)b, CTRL, ROWS, 0xF, false);
  const u32 hi = __builtin_amdgcn_update_dpp(0, (int)(u32)(b >> 32), CTRL, ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((u64)hi << 32) | lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_take<0xB1, 0xF>(v);   // quad_perm 1,0,3,2
  v += dpp_take<0x4E, 0xF>(v);   // quad_perm 2,3,0,1
  v += dpp_take<0x141, 0xF>(v);  // row_half_mirror
  v += dpp_take<0x140, 0xF>(v);  // row_mirror
  v += dpp_take<0x142, 0xA>(v);  // row_bcast 15, into rows 1 and 3
  v += dpp_take<0x143, 0xC>(v);  // row_bcast 31, into rows 2 and 3
  return v;
}
)";
  }
  if (perm) {
    // pi on a row or column index: the gate's local index l from its bits,
    // pi(l) from a packed table of 3-bit entries, the changed bits flipped.
    uint32_t pack = 0;
    for (int l = 0; l < (1 << perm->k); ++l) pack |= (uint32_t)perm->table[l] << (3 * l);
    add(s, "__device__ __forceinline__ u32 gate_l(u32 n) {\n  return 0u");
    for (int j = 0; j < perm->k; ++j) add(s, " | (((n >> %d) & 1u) << %d)", perm->bits[j], perm->k - 1 - j);
    add(s, ";\n}\n");
    add(s, "__device__ __forceinline__ u32 gate_perm(u32 n) {\n");
    add(s, "  const u32 l = gate_l(n), d = l ^ ((%uu >> (3u * l)) & 7u);\n  return n", pack);
    for (int j = 0; j < perm->k; ++j) add(s, " ^ (((d >> %d) & 1u) << %d)", perm->k - 1 - j, perm->bits[j]);
    add(s, ";\n}\n");
    if (!perm->unit) {
      // The phases u_l, exact (hexadecimal literals).  The conjugation's row
      // pass gives u x as one complex multiply-add from +0 (its other terms
      // are products with exact zeros), the column pass conj(u') times that:
      // the same operations here.
      add(s, "__device__ const double gate_ur[8] = {");
      for (int l = 0; l < 8; ++l) add(s, "%s%a", l ? ", " : "", perm->ur[l]);
      add(s, "};\n__device__ const double gate_ui[8] = {");
      for (int l = 0; l < 8; ++l) add(s, "%s%a", l ? ", " : "", perm->ui[l]);
      add(s, "};\n");
      s += R"(__device__ __forceinline__ double2 cmad0(double ux, double uy, double2 x) {
  double2 a = make_double2(0.0, 0.0);
  a.x = __fma_rn(ux, x.x, a.x);
  a.x = __fma_rn(-uy, x.y, a.x);
  a.y = __fma_rn(ux, x.y, a.y);
  a.y = __fma_rn(uy, x.x, a.y);
  return a;
}
)";
    }
  }
  if (low) add(s, "struct GateU { double v[%d]; };  // U row-major, (re, im) pairs\n", 2 * gm * gm);
  // (with the gate's passes the compiler would otherwise take a few VGPRs
  // past what three blocks per CU allow)
  add(s, "extern \"C\" __global__ __launch_bounds__(%d)%s void %s(const double2 *__restrict__ rho, "
         "double2 *__restrict__ out, const CT *__restrict__ tables, u32 *tickets, double p_keep, "
         "u32 xcd_blocks, u32 nsub%s%s) {\n", kTileThreads,
      low ? " __attribute__((amdgpu_waves_per_eu(3)))" : "", kSpecName,
      obs ? ", const double2 *__restrict__ psi0, double *__restrict__ part" : "",
      low ? ", const GateU gu" : "");
  if (low) {
    add(s, "  __shared__ double2 gx[%d];\n  __shared__ double2 gU[%d];\n", kTileElems, gm * gm);
    add(s, "  if (threadIdx.x < %du) gU[threadIdx.x] = make_double2(gu.v[2u * threadIdx.x], "
           "gu.v[2u * threadIdx.x + 1u]);\n", gm * gm);
  }
  if (G.own_staged) add(s, "  __shared__ double2 own_slot[%d];\n", kTileElems);
  if (G.any_staged) add(s, "  __shared__ double2 part_slot[%d];\n", kTileElems);
  if (G.tab_entries) {
    add(s, "  __shared__ CT tab[%zu];\n", G.tab_entries);
    add(s, "  for (u32 i = threadIdx.x; i < %zuu; i += %du) tab[i] = tables[i];\n", G.tab_entries,
        kTileThreads);
  }
  add(s, "  __shared__ u32 s_ticket[2];\n");
  add(s, "  const u32 tid = threadIdx.x, r = tid >> 4, c = tid & 15u;\n");
  add(s, "  const u32 t0b = ((r << %d) | c) << 4;\n", nq);
  for (int b = 0; b < 4; ++b) add(s, "  const u32 tf%d = (((r >> %d) & 1u) << 1) | ((c >> %d) & 1u);\n", b, b, b);
  add(s, "  const u32 x = blockIdx.x & 7u, sub = (blockIdx.x >> 3) %% nsub;\n");
  add(s, "  u32 *counter = tickets + (x * %uu + sub) * %uu;\n", kTicketSubs, kTicketStride);
  add(s, "  u32 drawn = 0;\n  if (tid == 0) drawn = atomicAdd(counter, 1u);\n");
  add(s, "  for (u32 it = 0;; ++it) {\n");
  add(s, "    if (tid == 0) s_ticket[it & 1u] = drawn * nsub + sub;\n    __syncthreads();\n");
  add(s, "    const u32 j = __builtin_amdgcn_readfirstlane(s_ticket[it & 1u]);\n");
  add(s, "    if (j >= %uu) break;\n", G.xcd_tiles);
  add(s, "    if (tid == 0) drawn = atomicAdd(counter, 1u);\n");
  // The thread's byte offset, made opaque for the tile: otherwise the
  // compiler hoists rho + t0b out of the loop and forms every address with a
  // 64-bit vector add, where (per-tile scalar base) + (32-bit vector offset)
  // needs none.
  add(s, "    u32 tv = t0b;\n    asm volatile(\"\" : \"+v\"(tv));\n");
  add(s, "    const u32 family = ((j >> %d) << 3) | x;\n", G.mb_bits);
  if (G.coset_order) {
    // A tile's partners differ from it by members in the span of the
    // partner flips.  With that span's basis first, the tiles of one coset
    // (closed under every flip) take consecutive tickets, so the partner
    // tiles in use on an XCD stay within a coset rather than the family.
    add(s, "    const u32 jm = j & %uu;\n    u32 nb = 0u", (1u << G.mb_bits) - 1u);
    for (int k = 0; k < G.mb_bits; ++k) add(s, " ^ (((jm >> %d) & 1u) * %uu)", k, G.member_basis[k]);
    add(s, ";\n    nb <<= 4;\n");
  } else {
    add(s, "    u32 nb = (j & %uu) << 4;\n", (1u << G.mb_bits) - 1u);
  }
  add(s, "    nb = ((nb >> %d) << %d) | (nb & %uu);\n", e0, e0 + 1, (1u << e0) - 1u);
  add(s, "    nb = ((nb >> %d) << %d) | (nb & %uu);\n", e1, e1 + 1, (1u << e1) - 1u);
  add(s, "    const u32 mb = nb ^ (family << 4);\n");
  add(s, "    const u64 u0 = (((u64)nb << %d) | mb) << 4;\n", nq);
  for (int b : ubits) add(s, "    const u32 uf%d = (((nb >> %d) & 1u) << 1) | ((mb >> %d) & 1u);\n", b, b, b);
  if (need_e0) add(s, "    const u32 fa0_0 = (mb >> %d) & 1u, fa0_1 = 2u | (fa0_0 ^ 1u);\n", e0);
  if (need_e1) add(s, "    const u32 fa1_0 = (mb >> %d) & 1u, fa1_1 = 2u | (fa1_0 ^ 1u);\n", e1);
  // byte offset of block b of a tile: (dep(b) << nq | dep(b)) * 16
  uint64_t db[4];
  for (int b = 0; b < 4; ++b) {
    const uint64_t d = ((b & 1) ? 1ull << e0 : 0) | ((b & 2) ? 1ull << e1 : 0);
    db[b] = ((d << nq) | d) << 4;
  }
  auto load = [&](const char *dst, uint64_t fb, int b, uint32_t lflob) {
    add(s, "    const double2 %s = *(const double2 *)((const char *)rho + (u0 ^ %lluull) + (tv ^ %uu));\n",
        dst, (unsigned long long)(fb ^ db[b]), lflob);
  };
  for (int a = 0; a < 4; ++a) {
    char nm[16];
    snprintf(nm, sizeof(nm), "own%d", a);
    load(nm, 0, a, 0);
  }
  const int np = (int)P.size();
  auto issue = [&](int p1) {
    for (int k = 0; k < kRound && p1 + k < np; ++k)
      for (int b = 0; b < 4; ++b) {
        char nm[24];
        snprintf(nm, sizeof(nm), "q%d_%d", p1 + k, b);
        load(nm, P[p1 + k].fRb, b, P[p1 + k].lflob);
      }
  };
  if (np > 1) issue(1);
  if (G.own_staged)
    for (int a = 0; a < 4; ++a) add(s, "    own_slot[%d + tid] = own%d;\n", a * 256, a);
  add(s, "    double2 acc0 = make_double2(0.0, 0.0), acc1 = acc0, acc2 = acc0, acc3 = acc0;\n");

  // Table index of segment rc for output a (a < 0: the segment avoids E0/E1).
  auto index = [&](const TRec &rc, int a) {
    std::string e;
    for (uint32_t j = 0; j < rc.nbits; ++j) {
      const int b = (int)((j == 0 ? rc.sh0 : j == 1 ? rc.sh1 : rc.sh2) / 2);
      char t[48];
      if (b < 4) snprintf(t, sizeof(t), "(tf%d << %u)", b, 2 * j);
      else if (b == e0) snprintf(t, sizeof(t), "(fa0_%d << %u)", a & 1, 2 * j);
      else if (b == e1) snprintf(t, sizeof(t), "(fa1_%d << %u)", (a >> 1) & 1, 2 * j);
      else snprintf(t, sizeof(t), "(uf%d << %u)", b, 2 * j);
      if (!e.empty()) e += " + ";
      e += t;
    }
    char t[48];
    snprintf(t, sizeof(t), "tab[%uu + ", rc.entry_b);
    return std::string(t) + e + "]";
  };
  auto process = [&](int p) {
    const TPartner &pt = P[p];
    add(s, "    {  // partner %d\n", p);
    if (pt.mode == kStaged) {
      add(s, "    __syncthreads();\n");
      for (int b = 0; b < 4; ++b) add(s, "    part_slot[%d + tid] = q%d_%d;\n", b * 256, p, b);
      add(s, "    __syncthreads();\n");
    } else if (pt.mode == kOwn && G.own_staged) {
      add(s, "    __syncthreads();\n");
    }
    for (uint32_t ri = pt.r_first; ri < pt.r_first + pt.r_count; ++ri) {
      const TRead &rd = R[ri];
      add(s, "    {  // read set f_lo*17 = %u\n", rd.flo17);
      for (int b = 0; b < 4; ++b) {
        if (pt.mode == kOwn && rd.flo17 == 0) add(s, "    const double2 v%d = own%d;\n", b, b);
        else if (pt.mode == kOwn) add(s, "    const double2 v%d = own_slot[%d + (tid ^ %uu)];\n", b, b * 256, rd.flo17);
        else if (pt.mode == kStaged) add(s, "    const double2 v%d = part_slot[%d + (tid ^ %uu)];\n", b, b * 256, rd.flo17);
        else add(s, "    const double2 v%d = q%d_%d;\n", b, p, b);
      }
      uint32_t ob = rd.rec;
      for (int kind = 0; kind < kKinds; ++kind) {
        const int fe = kind >> 1;
        const bool uni = (kind & 1) == 0;
        for (uint32_t g = 0; g < rd.count[kind]; ++g) {
          const TRec &first = S[ob];
          const uint32_t nseg = 1 + first.extra;
          add(s, "    {\n");
          if (uni) {
            add(s, "      CT cg = %s;\n", index(first, 0).c_str());
            for (uint32_t e = 1; e < nseg; ++e) add(s, "      cg = cadd(cg, %s);\n", index(S[ob + e], 0).c_str());
            for (int a = 0; a < 4; ++a) add(s, "      madd(acc%d, cg, v%d);\n", a, a ^ fe);
          } else {
            for (int a = 0; a < 4; ++a) add(s, "      CT c%d = %s;\n", a, index(first, a).c_str());
            for (uint32_t e = 1; e < nseg; ++e) {
              const TRec &sg = S[ob + e];
              if (sg.etouch) {
                for (int a = 0; a < 4; ++a) add(s, "      c%d = cadd(c%d, %s);\n", a, a, index(sg, a).c_str());
              } else {
                add(s, "      { const CT t = %s;\n", index(sg, 0).c_str());
                for (int a = 0; a < 4; ++a) add(s, "        c%d = cadd(c%d, t);\n", a, a);
                add(s, "      }\n");
              }
            }
            for (int a = 0; a < 4; ++a) add(s, "      madd(acc%d, c%d, v%d);\n", a, a, a ^ fe);
          }
          add(s, "    }\n");
          ob += nseg;
        }
      }
      add(s, "    }\n");
    }
    add(s, "    }\n");
  };
  process(0);
  for (int p1 = 1; p1 < np; p1 += kRound) {
    if (p1 > 1) issue(p1);
    for (int k = 0; k < kRound && p1 + k < np; ++k) process(p1 + k);
  }
  for (int a = 0; a < 4; ++a) {
    add(s, "    acc%d.x = __fma_rn(p_keep, own%d.x, acc%d.x);\n", a, a, a);
    add(s, "    acc%d.y = __fma_rn(p_keep, own%d.y, acc%d.y);\n", a, a, a);
  }
  if (low) {
    // The gate on bits 0..3 of n and m, which the tile's rows (r) and columns
    // (c) hold complete: as the conjugation computes it, first every row
    // group with U, then every column group with conj(U), each output a
    // chain of complex multiply-adds from +0 over the group's local index.
    // The tile's outputs pass through LDS between the two.
    auto dep = [&](int l) {  // bits of local index l at the gate's positions
      uint32_t d = 0;
      for (int j = 0; j < low->k; ++j)
        if ((l >> (low->k - 1 - j)) & 1) d |= 1u << low->bits[j];
      return d;
    };
    auto local = [&](int shift) {
      std::string e = "0u";
      for (int j = 0; j < low->k; ++j) {
        char b[64];
        snprintf(b, sizeof(b), " | (((tid >> %d) & 1u) << %d)", low->bits[j] + shift, low->k - 1 - j);
        e += b;
      }
      return e;
    };
    for (int a = 0; a < 4; ++a) add(s, "    gx[%du | tid] = acc%d;\n", a << 8, a);
    add(s, "    __syncthreads();\n    {\n");
    add(s, "      const u32 gl = (%s) * %du, gb = tid & %uu;\n", local(4).c_str(), gm, ~(gmask << 4) & 255u);
    for (int l = 0; l < gm; ++l) add(s, "      const double2 ur%d = gU[gl + %du];\n", l, l);
    for (int a = 0; a < 4; ++a) {
      add(s, "      acc%d = make_double2(0.0, 0.0);\n", a);
      for (int l = 0; l < gm; ++l)
        add(s, "      madd(acc%d, ur%d, gx[%uu | gb | %uu]);\n", a, l, (uint32_t)a << 8, dep(l) << 4);
    }
    add(s, "    }\n    __syncthreads();\n");
    for (int a = 0; a < 4; ++a) add(s, "    gx[%du | tid] = acc%d;\n", a << 8, a);
    add(s, "    __syncthreads();\n    {\n");
    add(s, "      const u32 gl = (%s) * %du, gb = tid & %uu;\n", local(0).c_str(), gm, ~gmask & 255u);
    for (int l = 0; l < gm; ++l)
      add(s, "      const double2 uc%d = make_double2(gU[gl + %du].x, -gU[gl + %du].y);\n", l, l, l);
    for (int a = 0; a < 4; ++a) {
      add(s, "      acc%d = make_double2(0.0, 0.0);\n", a);
      for (int l = 0; l < gm; ++l)
        add(s, "      madd(acc%d, uc%d, gx[%uu | gb | %uu]);\n", a, l, (uint32_t)a << 8, dep(l));
    }
    add(s, "    }\n");
  }
  if (obs) add(s, "    double o_tr = 0.0, o_ti = 0.0, o_pu = 0.0, o_fi = 0.0;\n");
  // Observables of the stored output w at (n2, m2): trace, sum |w|^2, and
  // Re conj(psi0[n2]) w psi0[m2], in a fixed order per thread.
  auto observe = [&](const char *n2, const char *m2) {
    if (!obs) return;
    add(s, "      if (%s == %s) { o_tr += w.x; o_ti += w.y; }\n", n2, m2);
    add(s, "      o_pu = __fma_rn(w.x, w.x, o_pu); o_pu = __fma_rn(w.y, w.y, o_pu);\n");
    if (obs < 2) return;
    if (nq + 4 <= 32)  // scalar base plus a 32-bit byte offset, no 64-bit address adds
      add(s, "      { const double2 pn = *(const double2 *)((const char *)psi0 + (%s << 4)),\n"
             "          pm = *(const double2 *)((const char *)psi0 + (%s << 4));\n", n2, m2);
    else
      add(s, "      { const double2 pn = psi0[%s], pm = psi0[%s];\n", n2, m2);
    add(s, "        const double tx = w.x * pm.x - w.y * pm.y, ty = w.x * pm.y + w.y * pm.x;\n");
    add(s, "        o_fi += pn.x * tx + pn.y * ty; }\n");
  };
  for (int a = 0; a < 4; ++a) {
    if (perm) {
      // output (n, m) of this thread goes to (pi(n), pi(m))
      const uint32_t d = ((a & 1) ? 1u << e0 : 0u) | ((a & 2) ? 1u << e1 : 0u);
      add(s, "    { const u32 n1 = nb | %uu | r, m1 = (mb ^ %uu) | c;\n", d, d);
      if (perm->unit) {
        add(s, "      const dbl2v w = {acc%d.x, acc%d.y};\n", a, a);
      } else {
        add(s, "      const u32 ln = gate_l(n1), lm = gate_l(m1);\n");
        add(s, "      const double2 t = cmad0(gate_ur[lm], -gate_ui[lm], cmad0(gate_ur[ln], gate_ui[ln], acc%d));\n", a);
        add(s, "      const dbl2v w = {t.x, t.y};\n");
      }
      add(s, "      const u32 n2 = gate_perm(n1), m2 = gate_perm(m1);\n");
      if (2 * nq + 4 <= 32)  // the byte offset fits 32 bits: scalar base plus a 32-bit offset
        add(s, "      __builtin_nontemporal_store(w, (dbl2v *)((char *)out + (((n2 << %d) | m2) << 4)));\n", nq);
      else
        add(s, "      __builtin_nontemporal_store(w, (dbl2v *)((char *)out + ((((u64)n2 << %d) | m2) << 4)));\n",
            nq);
      observe("n2", "m2");
      add(s, "    }\n");
    } else {
      const uint32_t d = ((a & 1) ? 1u << e0 : 0u) | ((a & 2) ? 1u << e1 : 0u);
      add(s, "    { const dbl2v w = {acc%d.x, acc%d.y};\n", a, a);
      add(s, "      __builtin_nontemporal_store(w, (dbl2v *)((char *)out + (u0 ^ %lluull) + tv));\n",
          (unsigned long long)db[a]);
      if (obs) add(s, "      const u32 n2 = nb | %uu | r, m2 = (mb ^ %uu) | c;\n", d, d);
      observe("n2", "m2");
      add(s, "    }\n");
    }
  }
  if (obs) {
    // The wave's sums (register moves between lanes, in a fixed order: lane
    // 63's total is the same on every call), one record of four per (tile,
    // wave) at a fixed place, so the final sum does not depend on which
    // block took which tile.
    add(s, "    o_tr = wave_sum(o_tr); o_ti = wave_sum(o_ti);\n");
    add(s, "    o_pu = wave_sum(o_pu); o_fi = wave_sum(o_fi);\n");
    add(s, "    if ((tid & 63u) == 63u) {\n");
    add(s, "      double *q = part + (((u64)x * %uull + j) * 4u + (tid >> 6)) * 4u;\n", G.xcd_tiles);
    add(s, "      q[0] = o_tr; q[1] = o_ti; q[2] = o_pu; q[3] = o_fi;\n    }\n");
  }
  add(s, "  }\n");
  add(s, "  u32 *done = tickets + (%uu + x) * %uu;\n", 8 * kTicketSubs, kTicketStride);
  add(s, "  if (tid == 0 && atomicAdd(done, 1u) == xcd_blocks - 1u) {\n");
  add(s, "    for (u32 k = 0; k < nsub; ++k) atomicExch(tickets + (x * %uu + k) * %uu, 0u);\n", kTicketSubs,
      kTicketStride);
  add(s, "    atomicExch(done, 0u);\n  }\n}\n");
  return s;
}

}  // namespace

namespace {

// A plan on the host: the descriptor and table bytes the generic kernel
// reads, their layout, and the source of the kernel specialised to it.
struct HostPlan {
  int e0 = 0, e1 = 0;
  bool real = false;
  TiledSummary sm{};
  int npartners = 0;
  size_t tab_entries = 0, tab_bytes = 0, tab_lds0 = 0;
  size_t o_p = 0, o_r = 0, o_s = 0, o_t = 0, o_k = 0;
  std::vector<unsigned char> bytes;  // descriptors, tables, zeroed ticket counters
  int64_t flops = 0;
  std::string src;
  // generator inputs (gen's vector pointers are set by whoever keeps them)
  GenPlan gen{};
  std::vector<TPartner> partners;
  std::vector<TRead> reads;
  std::vector<TRec> recs;  // entry_b: table entry index
};

// False when the channel does not suit the tiled kernel.
bool plan_host(int nq, const std::vector<std::pair<uint64_t, PermTerm>> &terms, HostPlan &H) {
  if (nq < kTiledMinQubits || nq > kTiledMaxQubits) return false;
  const uint32_t N = 1u << nq;
  std::map<uint32_t, std::vector<const PermTerm *>> by_flip;
  for (const auto &pr : terms) by_flip[(uint32_t)pr.first].push_back(&pr.second);

  // Tile bits: fewest partner tiles, then fewest read sets.
  int e0 = 4, e1 = 5;
  size_t best_p = SIZE_MAX, best_r = SIZE_MAX;
  for (int a = 4; a < nq; ++a)
    for (int b = a + 1; b < nq; ++b) {
      const uint32_t em = (1u << a) | (1u << b), rm = (N - 1) & ~(15u | em);
      std::set<uint32_t> ps = {0u}, rs;
      for (const auto &kv : by_flip) {
        ps.insert(kv.first & rm);
        rs.insert(kv.first & ~em);
      }
      if (ps.size() < best_p || (ps.size() == best_p && rs.size() < best_r)) {
        best_p = ps.size();
        best_r = rs.size();
        e0 = a;
        e1 = b;
      }
    }
  const uint32_t em = (1u << e0) | (1u << e1), rm = (N - 1) & ~(15u | em);
  auto on_e = [&](int b) { return b == e0 || b == e1; };

  // partner f_R -> f_lo -> f_E -> the group's hits
  std::map<uint32_t, std::map<uint32_t, std::map<int, const std::vector<const PermTerm *> *>>> plan;
  plan[0];
  for (const auto &kv : by_flip) {
    const uint32_t f = kv.first;
    const int fE = (int)((f >> e0) & 1u) | (int)(((f >> e1) & 1u) << 1);
    plan[f & rm][f & 15u][fE] = &kv.second;
  }
  std::vector<TPartner> partners;
  std::vector<TRead> reads;
  std::vector<TRec> recs;
  std::vector<double2> tab;
  TiledSummary sm{};
  sm.e0 = e0;
  sm.e1 = e1;
  int64_t flops_groups = 0, flops_segs = 0;
  for (const auto &pk : plan) {  // f_R ascending: the tile itself first
    TPartner P;
    memset(&P, 0, sizeof(P));
    P.fRb = (((uint64_t)pk.first << nq) | pk.first) << 4;
    P.r_first = (uint32_t)reads.size();
    P.r_count = (uint32_t)pk.second.size();
    for (const auto &lk : pk.second) {  // f_lo ascending
      TRead R;
      memset(&R, 0, sizeof(R));
      R.flo17 = lk.first * 17u;
      R.rec = (uint32_t)recs.size();
      for (int kind = 0; kind < kKinds; ++kind) {
        const int fE = kind >> 1;
        const bool uni = (kind & 1) == 0;
        auto it = lk.second.find(fE);
        if (it == lk.second.end()) continue;
        std::vector<SegBuild> sb = make_segments(*it->second);
        bool any_e = false;
        for (const SegBuild &sg : sb)
          for (int b : sg.bits) any_e = any_e || on_e(b);
        if (any_e == uni) continue;  // the group belongs to the other kind of its f_E
        // a group of the per-output kind starts with a segment on E0 or E1
        std::stable_partition(sb.begin(), sb.end(), [&](const SegBuild &sg) {
          return std::any_of(sg.bits.begin(), sg.bits.end(), on_e);
        });
        for (size_t si = 0; si < sb.size(); ++si) {
          const SegBuild &sg = sb[si];
          TRec S;
          memset(&S, 0, sizeof(S));
          const int nb = (int)sg.bits.size();
          S.sh0 = 2 * sg.bits[0];
          S.sh1 = nb > 1 ? 2 * sg.bits[1] : kZeroField;
          S.sh2 = nb > 2 ? 2 * sg.bits[2] : kZeroField;
          S.entry_b = (uint32_t)tab.size();  // the entry; made an LDS byte address below
          S.nbits = (uint32_t)nb;
          for (int b : sg.bits) S.etouch |= on_e(b) ? 1u : 0u;
          S.extra = si == 0 ? (uint32_t)(sb.size() - 1) : 0u;
          const std::vector<double2> t = segment_table(sg);
          tab.insert(tab.end(), t.begin(), t.end());
          sm.etouch_segments += (int)S.etouch;
          ++sm.segments;
          recs.push_back(S);
        }
        ++R.count[kind];
        R.kinds |= 1u << kind;
        flops_segs += (int64_t)sb.size() - 1;
        ++flops_groups;
        ++sm.groups;
      }
      reads.push_back(R);
    }
    if (partners.empty()) {
      P.mode = kOwn;
      for (const auto &lk : pk.second) sm.own_staged |= lk.first != 0 ? 1 : 0;
    } else {
      P.mode = P.r_count >= 2 ? kStaged : kDirect;
      (P.mode == kStaged ? sm.staged : sm.direct) += 1;
      if (P.mode == kDirect) {
        const uint64_t f = pk.second.begin()->first;
        P.lflob = (uint32_t)(((f << nq) | f) << 4);
      }
    }
    partners.push_back(P);
  }
  bool real = true;
  for (const double2 &v : tab) real = real && v.y == 0.0;
  const size_t tab_bytes = tab.size() * (real ? sizeof(double) : sizeof(double2));
  if (tab_bytes > kTableBytesMax) return false;
  sm.partners = (int)partners.size();
  sm.reads = (int)reads.size();
  sm.real = real ? 1 : 0;
  GenPlan gp;
  gp.nq = nq;
  gp.e0 = e0;
  gp.e1 = e1;
  gp.mb_bits = nq - 6;
  gp.xcd_tiles = 1u << (2 * nq - 13);
  gp.real = real;
  gp.own_staged = sm.own_staged != 0;
  gp.any_staged = sm.staged > 0;
  gp.tab_entries = tab.size();
  // Member-space vectors of the partner flips (tile base bits 4.. without
  // E0, E1, packed), a basis of their span first, then unit vectors.
  {
    std::vector<int> pos;
    for (int b = 4; b < nq; ++b)
      if (b != e0 && b != e1) pos.push_back(b);
    const int mbits = (int)pos.size();  // == nq - 6
    std::vector<uint32_t> basis, reduced;  // reduced: echelon copies for the rank test
    auto try_add = [&](uint32_t v) {
      uint32_t w = v;
      for (uint32_t r : reduced)
        if ((w ^ r) < w) w ^= r;  // r's leading bit is set in w: clear it
      if (!w) return;
      basis.push_back(v);
      reduced.push_back(w);
      std::sort(reduced.begin(), reduced.end(), std::greater<uint32_t>());
    };
    for (const auto &pk : plan) {
      uint32_t h = 0;
      for (int i = 0; i < mbits; ++i) h |= ((pk.first >> pos[i]) & 1u) << i;
      if (h) try_add(h);
    }
    const size_t rank = basis.size();
    for (int i = 0; i < mbits; ++i) try_add(1u << i);
    gp.coset_order = rank < (size_t)mbits;
    for (int k = 0; k < mbits && k < 32; ++k) gp.member_basis[k] = basis[k];
  }
  gp.partners = &partners;
  gp.reads = &reads;
  gp.recs = &recs;
  const std::string spec_src = tiled_source(gp, nullptr, 0);
  H.gen = gp;
  H.partners = partners;
  H.reads = reads;
  H.recs = recs;
  // LDS: the own tile (when staged), the staged partner, then the tables.
  const size_t tab_lds0 = (sm.own_staged ? kTileElems * sizeof(double2) : 0) +
                          (sm.staged ? kTileElems * sizeof(double2) : 0);
  for (TRec &S : recs)
    S.entry_b = (uint32_t)(tab_lds0 + S.entry_b * (real ? sizeof(double) : sizeof(double2)));

  const size_t o_p = 0, o_r = align256(o_p + sizeof(TPartner) * partners.size());
  const size_t o_s = align256(o_r + sizeof(TRead) * reads.size());
  const size_t o_t = align256(o_s + sizeof(TRec) * recs.size());
  const size_t o_k = align256(o_t + tab_bytes);
  const size_t total = o_k + (8 * kTicketSubs + 8) * kTicketStride * sizeof(uint32_t);  // zero
  std::vector<unsigned char> host(total, 0);
  memcpy(host.data() + o_p, partners.data(), sizeof(TPartner) * partners.size());
  if (!reads.empty()) memcpy(host.data() + o_r, reads.data(), sizeof(TRead) * reads.size());
  if (!recs.empty()) memcpy(host.data() + o_s, recs.data(), sizeof(TRec) * recs.size());
  for (size_t i = 0; i < tab.size(); ++i) {
    if (real)
      memcpy(host.data() + o_t + i * sizeof(double), &tab[i].x, sizeof(double));
    else
      memcpy(host.data() + o_t + i * sizeof(double2), &tab[i], sizeof(double2));
  }
  H.e0 = e0;
  H.e1 = e1;
  H.real = real;
  H.sm = sm;
  H.npartners = (int)partners.size();
  H.tab_entries = tab.size();
  H.tab_bytes = tab_bytes;
  H.tab_lds0 = tab_lds0;
  H.o_p = o_p;
  H.o_r = o_r;
  H.o_s = o_s;
  H.o_t = o_t;
  H.o_k = o_k;
  H.bytes = std::move(host);
  H.flops = 2 + flops_groups * (real ? 4 : 8) + flops_segs * (real ? 1 : 2);
  H.src = spec_src;
  return true;
}

}  // namespace

std::string tiled_channel_source(int nq, const std::vector<std::pair<uint64_t, PermTerm>> &terms,
                                 const OutPerm *perm, bool obs) {
  HostPlan H;
  if (!plan_host(nq, terms, H)) return std::string();
  if (!perm && !obs) return H.src;
  H.gen.partners = &H.partners;
  H.gen.reads = &H.reads;
  H.gen.recs = &H.recs;
  return tiled_source(H.gen, perm, obs ? 2 : 0);
}

int tiled_channel_compile_check(const std::string &src, size_t *code_bytes) {
  return rtc_compile(src, kSpecName, code_bytes);
}

int tiled_channel_compiler_version() { return rtc_compiler_version(); }

namespace {

// Persistent grid of a compiled kernel: resident blocks (capped per CU, see
// spec_blocks_per_cu) over the device, a multiple of the 8 XCDs.
bool spec_launch(const TiledChannel *t, const RtcKernel *k, TiledChannel::Launch *ls) {
  int bpc = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, k->fn, kTileThreads, 0) != hipSuccess ||
      k->num_regs <= 0) {
    (void)hipGetLastError();
    return false;
  }
  bpc = std::min(bpc, std::min(spec_blocks_per_cu(t->args.nq), 512 / ((k->num_regs + 7) / 8 * 8)));
  if (bpc < 1) return false;
  const uint64_t want = std::min<uint64_t>((uint64_t)bpc * t->ncu, (uint64_t)t->args.xcd_tiles * 8);
  ls->k = k;
  ls->grid = (unsigned)std::max<uint64_t>(8, want & ~(uint64_t)7);
  ls->xcd_blocks = ls->grid / 8;
  ls->nsub = ticket_subs(ls->xcd_blocks);
  return true;
}

int launch_spec(const TiledChannel *t, const TiledChannel::Launch &ls, const double2 *in, double2 *out,
                hipStream_t s, const double2 *psi0 = nullptr, double *part = nullptr,
                const double *gate_u = nullptr) {
  const double2 *a_in = in;
  double2 *a_out = out;
  const void *a_tab = t->args.tables;
  uint32_t *a_tk = t->args.tickets;
  double a_p = t->args.p_keep;
  uint32_t a_xb = ls.xcd_blocks, a_ns = ls.nsub;
  const double2 *a_psi = psi0;
  double *a_part = part;
  double a_gu[128];  // the gate's matrix, passed by value
  void *args[10] = {&a_in, &a_out, &a_tab, &a_tk, &a_p, &a_xb, &a_ns};
  int n = 7;
  if (ls.obs) {
    args[n++] = &a_psi;
    args[n++] = &a_part;
  }
  if (ls.gate_words) {
    if (!gate_u) return fail(QCW_EINVAL, "the folded gate's matrix is missing");
    memcpy(a_gu, gate_u, sizeof(double) * (size_t)ls.gate_words);
    args[n++] = a_gu;
  }
  if (hipModuleLaunchKernel(ls.k->fn, ls.grid, 1, 1, kTileThreads, 1, 1, 0, s, args, nullptr) !=
      hipSuccess)
    return fail(QCW_EHIP, "channel launch: %s", hipGetErrorString(hipGetLastError()));
  return QCW_OK;
}

// The compiled kernel variant for a folded gate (p, or none) and with or
// without observables (compiled on first use), or nullptr.
const TiledChannel::Launch *variant_launch(const TiledChannel *t, const OutPerm *p, int obs) {
  if (!t->spec) return nullptr;
  std::vector<int> key = {obs, p ? p->k : 0, p ? p->general : 0};
  for (int j = 0; p && j < p->k; ++j) key.push_back(p->bits[j]);
  for (int l = 0; p && l < (1 << p->k); ++l) {
    key.push_back(p->table[l]);
    for (const double v : {p->ur[l], p->ui[l]}) {
      int32_t w[2];
      memcpy(w, &v, sizeof(v));
      key.push_back(w[0]);
      key.push_back(w[1]);
    }
  }
  std::lock_guard<std::mutex> lk(t->perm_mu);
  auto it = t->perm_kernels.find(key);
  if (it != t->perm_kernels.end()) return it->second.k ? &it->second : nullptr;
  TiledChannel::Launch ls;
  const RtcKernel *k = nullptr;
  if (rtc_get(tiled_source(t->gen, p, obs), kSpecName, &k) != QCW_OK || !spec_launch(t, k, &ls)) {
    ls = {};
  } else {
    ls.obs = obs;
    ls.gate_words = p && p->general ? 2 << (2 * p->k) : 0;
  }
  clear_error();
  auto &e = t->perm_kernels[key];
  e = ls;
  return e.k ? &e : nullptr;
}

}  // namespace

bool tiled_channel_perm_ready(const TiledChannel *t, const OutPerm &perm) {
  return t && variant_launch(t, &perm, 0) != nullptr;
}

int tiled_channel_apply_perm(const TiledChannel *t, const OutPerm &perm, const double2 *in,
                             double2 *out, hipStream_t s, const double *gate_u) {
  const TiledChannel::Launch *ls = t ? variant_launch(t, &perm, 0) : nullptr;
  if (!ls) return QCW_EAGAIN;
  return launch_spec(t, *ls, in, out, s, nullptr, nullptr, gate_u);
}

bool tiled_channel_obs_ready(const TiledChannel *t, const OutPerm *perm, bool fidelity) {
  return t && variant_launch(t, perm, fidelity ? 2 : 1) != nullptr;
}

uint64_t tiled_channel_obs_records(const TiledChannel *t) {
  return t ? (uint64_t)t->args.xcd_tiles * 8u * 4u : 0;
}

int tiled_channel_apply_obs(const TiledChannel *t, const OutPerm *perm, const double2 *in,
                            double2 *out, const double2 *psi0, double *part, hipStream_t s,
                            const double *gate_u) {
  const TiledChannel::Launch *ls = t ? variant_launch(t, perm, psi0 ? 2 : 1) : nullptr;
  if (!ls) return QCW_EAGAIN;
  return launch_spec(t, *ls, in, out, s, psi0, part, gate_u);
}

int tiled_channel_create(int nq, double p_keep,
                         const std::vector<std::pair<uint64_t, PermTerm>> &terms,
                         TiledChannel **out) {
  *out = nullptr;
  HostPlan H;
  if (!plan_host(nq, terms, H)) return QCW_OK;
  const size_t total = H.bytes.size();
  TiledChannel *t = new TiledChannel();
  t->real = H.real;
  t->sum = H.sm;
  t->lds = H.tab_lds0 + H.tab_bytes;
  t->flops = H.flops;
  if (hipMalloc(&t->dbuf, total) != hipSuccess ||
      hipMemcpy(t->dbuf, H.bytes.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    tiled_channel_free(t);
    return fail(QCW_ENOMEM, "channel plan upload failed");
  }
  const bool real = H.real;
  unsigned char *d = static_cast<unsigned char *>(t->dbuf);
  TArgs &A = t->args;
  A.nq = nq;
  A.e0 = H.e0;
  A.e1 = H.e1;
  A.mb_bits = nq - 6;
  A.p_keep = p_keep;
  A.xcd_tiles = 1u << (2 * nq - 13);
  A.npartners = H.npartners;
  A.own_staged = H.sm.own_staged;
  A.any_staged = H.sm.staged > 0 ? 1 : 0;
  A.tab_entries = (int)H.tab_entries;
  A.partners = reinterpret_cast<const TPartner *>(d + H.o_p);
  A.reads = reinterpret_cast<const TRead *>(d + H.o_r);
  A.recs = reinterpret_cast<const TRec *>(d + H.o_s);
  A.tables = d + H.o_t;
  A.tickets = reinterpret_cast<uint32_t *>(d + H.o_k);

  // Persistent grid: resident blocks over the device, a multiple of the 8
  // XCDs so that a block keeps its XCD's families.
  int dev = 0, bpc = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, tiled_fn(real), kTileThreads, t->lds) !=
          hipSuccess ||
      hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    tiled_channel_free(t);
    return fail(QCW_EHIP, "channel occupancy query failed");
  }
  // Blocks beyond those resident would start only as others finish their
  // share, a tail on an idle device: bound the query by the register file
  // too (512 VGPRs per lane and SIMD in granules of 8; a block is one wave
  // per SIMD).
  hipFuncAttributes fa;
  if (hipFuncGetAttributes(&fa, tiled_fn(real)) == hipSuccess && fa.numRegs > 0) {
    bpc = std::min(bpc, std::min(8, 512 / ((fa.numRegs + 7) / 8 * 8)));
    t->sum.regs = fa.numRegs;
  }
  (void)hipGetLastError();
  if (bpc < 1) {
    tiled_channel_free(t);
    return QCW_OK;
  }
  const uint64_t want = std::min<uint64_t>((uint64_t)bpc * ncu, (uint64_t)A.xcd_tiles * 8);
  t->grid = (unsigned)std::max<uint64_t>(8, want & ~(uint64_t)7);
  A.xcd_blocks = t->grid / 8;
  A.nsub = ticket_subs(A.xcd_blocks);

  // The kernel compiled for this plan; without it the generic kernel runs.
  t->g_partners = std::move(H.partners);
  t->g_reads = std::move(H.reads);
  t->g_recs = std::move(H.recs);
  t->gen = H.gen;
  t->gen.partners = &t->g_partners;
  t->gen.reads = &t->g_reads;
  t->gen.recs = &t->g_recs;
  t->ncu = ncu;
  const RtcKernel *k = nullptr;
  TiledChannel::Launch ls;
  if (rtc_get(H.src, kSpecName, &k) == QCW_OK && spec_launch(t, k, &ls)) {
    t->spec = k;
    t->spec_grid = ls.grid;
    t->spec_xcd_blocks = ls.xcd_blocks;
    t->spec_nsub = ls.nsub;
  }
  t->sum.specialized = t->spec ? 1 : 0;
  t->sum.grid = (int)t->grid;
  t->sum.spec_grid = (int)t->spec_grid;
  t->sum.spec_regs = k ? k->num_regs : 0;
  clear_error();
  *out = t;
  return QCW_OK;
}

int tiled_channel_apply(const TiledChannel *t, const double2 *in, double2 *out, hipStream_t s,
                        bool generic) {
  if (t->spec && !generic) {
    TiledChannel::Launch ls;
    ls.k = t->spec;
    ls.grid = t->spec_grid;
    ls.xcd_blocks = t->spec_xcd_blocks;
    ls.nsub = t->spec_nsub;
    return launch_spec(t, ls, in, out, s);
  }
  if (t->real)
    hipLaunchKernelGGL(channel_tiled_kernel<true>, dim3(t->grid), dim3(kTileThreads), t->lds, s, in,
                       out, t->args);
  else
    hipLaunchKernelGGL(channel_tiled_kernel<false>, dim3(t->grid), dim3(kTileThreads), t->lds, s,
                       in, out, t->args);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(QCW_EHIP, "channel launch: %s", hipGetErrorString(e));
  return QCW_OK;
}

void tiled_channel_free(TiledChannel *t) {
  if (!t) return;
  (void)hipFree(t->dbuf);
  delete t;
}

int64_t tiled_channel_flops(const TiledChannel *t) { return t ? t->flops : 0; }

void tiled_channel_summary(const TiledChannel *t, TiledSummary *s) {
  if (t) *s = t->sum;
}

}  // namespace qcw

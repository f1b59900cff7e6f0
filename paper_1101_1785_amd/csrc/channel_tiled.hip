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
#include <string.h>

#include <algorithm>
#include <map>
#include <set>
#include <vector>

#include "channel_tiled.h"
#include "qcw_common.h"

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
  // tile's work.
  const uint32_t x = blockIdx.x & 7u;
  const uint32_t sub = (blockIdx.x >> 3) % A.nsub;
  uint32_t *counter = A.tickets + (x * kTicketSubs + sub) * kTicketStride;
  __shared__ uint32_t s_ticket[2];
  uint32_t next = 0;
  if (threadIdx.x == 0) next = atomicAdd(counter, 1u) * A.nsub + sub;
  for (uint32_t it = 0;; ++it) {
    if (threadIdx.x == 0) s_ticket[it & 1u] = next;
    // Also the tile-start barrier: the previous tile's LDS reads are done
    // (first time: tables copied).  The ticket slot alternates, so the next
    // one cannot overwrite one still being read.
    __syncthreads();
    const uint32_t j = s_ticket[it & 1u];
    if (j >= A.xcd_tiles) break;
    if (threadIdx.x == 0) next = atomicAdd(counter, 1u) * A.nsub + sub;
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

}  // namespace

int tiled_channel_create(int nq, double p_keep,
                         const std::vector<std::pair<uint64_t, PermTerm>> &terms,
                         TiledChannel **out) {
  *out = nullptr;
  if (nq < kTiledMinQubits || nq > kTiledMaxQubits) return QCW_OK;
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
  if (tab_bytes > kTableBytesMax) return QCW_OK;
  sm.partners = (int)partners.size();
  sm.reads = (int)reads.size();
  sm.real = real ? 1 : 0;
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

  TiledChannel *t = new TiledChannel();
  t->real = real;
  t->sum = sm;
  t->lds = tab_lds0 + tab_bytes;
  t->flops = 2 + flops_groups * (real ? 4 : 8) + flops_segs * (real ? 1 : 2);
  if (hipMalloc(&t->dbuf, total) != hipSuccess ||
      hipMemcpy(t->dbuf, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipGetLastError();
    tiled_channel_free(t);
    return fail(QCW_ENOMEM, "channel plan upload failed");
  }
  unsigned char *d = static_cast<unsigned char *>(t->dbuf);
  TArgs &A = t->args;
  A.nq = nq;
  A.e0 = e0;
  A.e1 = e1;
  A.mb_bits = nq - 6;
  A.p_keep = p_keep;
  A.xcd_tiles = 1u << (2 * nq - 13);
  A.npartners = (int)partners.size();
  A.own_staged = sm.own_staged;
  A.any_staged = sm.staged > 0 ? 1 : 0;
  A.tab_entries = (int)tab.size();
  A.partners = reinterpret_cast<const TPartner *>(d + o_p);
  A.reads = reinterpret_cast<const TRead *>(d + o_r);
  A.recs = reinterpret_cast<const TRec *>(d + o_s);
  A.tables = d + o_t;
  A.tickets = reinterpret_cast<uint32_t *>(d + o_k);

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
  if (hipFuncGetAttributes(&fa, tiled_fn(real)) == hipSuccess && fa.numRegs > 0)
    bpc = std::min(bpc, std::min(8, 512 / ((fa.numRegs + 7) / 8 * 8)));
  (void)hipGetLastError();
  if (bpc < 1) {
    tiled_channel_free(t);
    return QCW_OK;
  }
  const uint64_t want = std::min<uint64_t>((uint64_t)bpc * ncu, (uint64_t)A.xcd_tiles * 8);
  t->grid = (unsigned)std::max<uint64_t>(8, want & ~(uint64_t)7);
  A.xcd_blocks = t->grid / 8;
  A.nsub = 1;
  while (A.nsub < kTicketSubs && 2 * A.nsub <= A.xcd_blocks) A.nsub *= 2;
  *out = t;
  return QCW_OK;
}

int tiled_channel_apply(const TiledChannel *t, const double2 *in, double2 *out, hipStream_t s) {
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

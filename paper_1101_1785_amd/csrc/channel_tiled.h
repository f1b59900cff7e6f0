// Permutation-type channel terms and the tiled channel kernel (channel_tiled.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

namespace qcw {

// A term whose operators each have one nonzero entry per row, in distinct
// columns (Pauli operators, phases, the identity): row r of K reads column
// r ^ s with s = 0 or 1, so (K rho K^dagger)_{nm} = c(n, m) rho_{n^x, m^x}
// with x the term's flip mask (the bits of its swapping operators) and
// c = K[r][r^s] conj(K[c][c^s]) depending only on the bits at the term's qubits.
struct PermTerm {
  int32_t nops;
  int32_t bit0, bit1;
  int32_t pad;
  double2 c0[4];  // w K0[r][r^s0] conj(K0[c][c^s0]) at r*2 + c (weight folded in)
  double2 c1[4];  // K1[r][r^s1] conj(K1[c][c^s1]) at r*2 + c
};

// Bit b of x (b < 16) moved to bit 2b.
__device__ __forceinline__ uint32_t spread16(uint32_t x) {
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

constexpr int kTiledMinQubits = 7;   // low 4 bits, two tile bits, at least one more
constexpr int kTiledMaxQubits = 15;  // row and column bits interleave into bits 0..29

struct TiledChannel;

// A monomial gate (one nonzero entry in each row and column: permutations
// such as X, CNOT, SWAP, Toffoli, times phases, such as Z, S, T, Y, CZ) on the
// state bits bits[0..k-1] (argument order: bits[0] is the most significant
// bit of the local index l): U |l> = u_l |pi(l)>, table[l] = pi(l).  The
// conjugation rho -> U rho U^dagger moves element (n, m) to (pi(n), pi(m))
// and multiplies it by u_l(n) conj(u_l(m)).
//
// With general set, the gate is any k-qubit matrix on bits among 0..3 (the
// four lowest qubits), whose rows and columns a tile holds complete: the
// kernel applies it to the tile's outputs in LDS, and its matrix (gate_u
// below: m x m, row-major, (re, im) pairs) arrives with each launch, so one
// compiled kernel serves every matrix on those qubits.  table, ur, ui and
// unit are then unused.
struct OutPerm {
  int k;
  int bits[3];
  uint8_t table[8];
  double ur[8], ui[8];  // u_l
  int unit;             // every u_l is exactly 1: a plain permutation
  int general;          // a general gate on bits 0..3 (see above)
};

// Shape of a tiled plan (for tests and reports).
struct TiledSummary {
  int e0, e1;          // the two tile bits above bit 3
  int partners;        // partner tiles per tile, the tile itself included
  int staged, direct;  // partners staged in LDS, partners read directly
  int own_staged;      // the tile itself staged in LDS (a flip inside it moves bits 0..3)
  int reads, groups, segments, etouch_segments;
  int real;            // every combined coefficient is real (2 FMAs per group and output)
  int specialized;     // a kernel compiled for this plan at run time is available
  int grid, regs;            // the generic kernel's persistent grid and VGPRs per lane
  int spec_grid, spec_regs;  // the same for the compiled kernel
};

// Plans the tiled form of a channel whose terms are all permutation type,
// given as (flip mask, term), and compiles the tiled kernel specialised to the
// plan (the generic kernel, which reads the plan from memory, serves when the
// run-time compiler is unavailable).  Returns QCW_OK with *out == nullptr
// when the channel does not suit it (nq outside [kTiledMinQubits,
// kTiledMaxQubits], coefficient tables beyond the LDS budget); an error code
// only when device memory cannot be had.
int tiled_channel_create(int nq, double p_keep,
                         const std::vector<std::pair<uint64_t, PermTerm>> &terms,
                         TiledChannel **out);
// generic: run the generic kernel even when a specialised one is compiled.
int tiled_channel_apply(const TiledChannel *t, const double2 *in, double2 *out, hipStream_t s,
                        bool generic);
void tiled_channel_free(TiledChannel *t);
// Source of the kernel specialised to the plan of these terms, storing its
// outputs at their places after the monomial gate `perm` when it is not
// NULL, and summing the observables when obs (host only; empty when the
// channel does not suit the tiled kernel).
std::string tiled_channel_source(int nq, const std::vector<std::pair<uint64_t, PermTerm>> &terms,
                                 const OutPerm *perm = nullptr, bool obs = false);
// The channel followed by conjugation with a monomial gate, in one pass:
// the compiled kernel stores output (n, m), times u_l(n) conj(u_l(m)), at
// (pi(n), pi(m)).  The kernel for
// each gate is compiled on first use.  QCW_EAGAIN when no compiled kernel is
// available (the caller then applies the channel and the gate separately).
int tiled_channel_apply_perm(const TiledChannel *t, const OutPerm &perm, const double2 *in,
                             double2 *out, hipStream_t s, const double *gate_u = nullptr);
// Whether tiled_channel_apply_perm would run (compiling the kernel if needed).
bool tiled_channel_perm_ready(const TiledChannel *t, const OutPerm &perm);
// The same kernels (perm may be NULL: no gate) that also reduce the stored
// rho's trace (re, im), sum |rho|^2 and Re <psi0|rho|psi0> (psi0: device,
// 2^nq amplitudes, or NULL): each wave writes its four sums for its part
// of a tile to part, at a place fixed by the tile (tiled_channel_obs_records
// records of four doubles), to be summed in a fixed order.  QCW_EAGAIN when
// no compiled kernel is available.
int tiled_channel_apply_obs(const TiledChannel *t, const OutPerm *perm, const double2 *in,
                            double2 *out, const double2 *psi0, double *part, hipStream_t s,
                            const double *gate_u = nullptr);
bool tiled_channel_obs_ready(const TiledChannel *t, const OutPerm *perm, bool fidelity);
uint64_t tiled_channel_obs_records(const TiledChannel *t);
// Compiles such a source for gfx950 without loading it (no device needed);
// sets the code object's size.
int tiled_channel_compile_check(const std::string &src, size_t *code_bytes);
// Version of the run-time compiler, major * 100 + minor (0: unavailable).
int tiled_channel_compiler_version();
// Real FP64 operations per output element, as the tiled kernel evaluates them.
int64_t tiled_channel_flops(const TiledChannel *t);
void tiled_channel_summary(const TiledChannel *t, TiledSummary *s);

}  // namespace qcw

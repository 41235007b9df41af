// Internal device descriptors shared by the host planner (fc_plan.cpp) and the
// gfx950 kernels (fc_kernels.hip). Plain POD structs, 8-byte aligned.
#pragma once
#include <stdint.h>

namespace fcx {

// Largest transform handled in one workgroup: 256 threads x 16 complex values.
constexpr int kThreads = 256;
constexpr int kMaxPoints = 4096;
constexpr int kTwiddleN = 4096;      // global twiddle table: exp(-j 2 pi k / 4096)
constexpr int kRxMaxDest = 4;        // RX: LDS destinations per long-FFT bin
constexpr int kRxMaxLds = 8192;      // RX: LDS entries available to one group's subband regions

enum IoType : int32_t { IO_C64 = 0, IO_F16 = 1, IO_BF16 = 2 };

// LDS slots of a transform buffer of n points (one pad slot per 32, see
// the device code's pad()).
constexpr int lds_elems(int n) { return n + (n >> 5); }

// Transform sizes: powers of two 16..4096, and the mixed-radix sizes
// 3 x 2^k for 768..3072 (three decimated 2^k-point transforms and a radix-3
// combination; the paper's example of a short transform of 768 = 3 x 256
// points, Sec. VI-C). Interpolation factors n_long / n_short are powers of two.
constexpr bool is_pow2c(int v) { return v > 0 && (v & (v - 1)) == 0; }
constexpr bool is_tri(int P) { return P % 3 == 0 && is_pow2c(P / 3) && P >= 768 && P <= 3072; }
constexpr bool fft_size_ok(int P) { return (is_pow2c(P) && P >= 16 && P <= kMaxPoints) || is_tri(P); }
// entries of the radix-3 combination's twiddle table exp(-j 2 pi k / 3072),
// stored after the per-pass twiddle bases (every 3 x 2^k size divides 3072)
constexpr int kTw3N = 3072;
// a group of long size N holds subbands of size L when N / L is an integral power of two
constexpr bool divides_pow2(int L, int N) { return L <= N && N % L == 0 && is_pow2c(N / L); }

// TX pruned kernel. Short FFTs one per wave (blocks in groups, one band
// region each) for L < 256 and for N <= 1024; otherwise on the whole
// workgroup in the long IFFT buffer, one block at a time: that frees the
// band regions' LDS, and the extra workgroups per CU outweigh the smaller
// per-wave transforms (measured on the batched TX: 2.07 against 2.27 ms).
// Grouped blocks: LDS = long IFFT buffer, OLA carry, one band region per
// block; four or three blocks where that lets three workgroups share a CU
// (one idle wave in the short-FFT phase costs less than a third workgroup
// gains), else the most of {4, 2, 1} that lets two share it.
//
// Transform plans (tuning, chosen by the autotuner): plan 0 takes the rule
// above; plan 1 the other placement of the short FFTs where both exist
// (L <= 1024). For the RX family plan 1 takes the long FFT with the next
// lower radix cap (radix 8 passes at N = 4096, radix 4 at N = 2048).
constexpr int pruned_lds_entries(int L, int N, int nb) { return lds_elems(N) + N / 2 + nb * lds_elems(L); }
constexpr bool pruned_wave_short(int L, int N) { return L < 256 || (L <= 1024 && N < 2048); }
constexpr bool pruned_ws(int L, int N, int tp) {
  return tp == 0 ? pruned_wave_short(L, N) : (L <= 1024 && !pruned_wave_short(L, N));
}
constexpr bool pruned_has_alt(int L) { return L <= 1024; }
constexpr int pruned_group_blocks(int L, int N, int tp = 0) {
  return !pruned_ws(L, N, tp) ? 1
         : pruned_lds_entries(L, N, 4) * 8 <= 163840 / 3 ? 4
         : pruned_lds_entries(L, N, 3) * 8 <= 163840 / 3 ? 3
         : pruned_lds_entries(L, N, 4) * 8 <= 80 * 1024 ? 4
         : pruned_lds_entries(L, N, 2) * 8 <= 80 * 1024 ? 2 : 1;
}
constexpr int pruned_lds_bytes(int L, int N, int tp = 0) {
  return pruned_lds_entries(L, N, pruned_ws(L, N, tp) ? pruned_group_blocks(L, N, tp) : 0) * 8;
}
// Workgroups per CU that the LDS allows (160 KiB per CU), at most three: the
// register budget follows, so that registers do not lower the occupancy the
// LDS allows, without forcing spills where LDS would allow four.
constexpr int pruned_waves_per_simd(int L, int N, int tp = 0) {
  return 163840 / pruned_lds_bytes(L, N, tp) >= 3 ? 3 : 163840 / pruned_lds_bytes(L, N, tp);
}

// Demodulating RX: waves per SIMD that the kernel's register budget keeps
// (its launch bounds). The second-block terms live in a second LDS region set
// where the LDS of the two sets still lets that many workgroups share a CU
// (a workgroup is one wave per SIMD), else in per-task device scratch.
constexpr int rxd_waves_per_simd(int io) { return io == IO_C64 ? 2 : 3; }
constexpr bool rxd_terms_in_lds(int io, int lds_two_sets_bytes) {
  return 163840 / lds_two_sets_bytes >= rxd_waves_per_simd(io);
}

// Weight gradient of a one-subband group with L <= 1024, blocks in groups:
// long-FFT buffer, then per block of a group its band region and its
// short-FFT buffer (the per-bin sums are held in registers); the most of
// {4, 2, 1} blocks that lets three workgroups share a CU, else the most
// within 80 KiB (two workgroups).
constexpr int wgg_lds_entries(int L, int N, int nb) { return lds_elems(N) + 2 * nb * lds_elems(L); }
constexpr int wgg_group_blocks(int L, int N) {
  return wgg_lds_entries(L, N, 4) * 8 <= 163840 / 3 ? 4
         : wgg_lds_entries(L, N, 2) * 8 <= 163840 / 3 ? 2
         : wgg_lds_entries(L, N, 1) * 8 <= 163840 / 3 ? 1
         : wgg_lds_entries(L, N, 4) * 8 <= 80 * 1024 ? 4 : wgg_lds_entries(L, N, 2) * 8 <= 80 * 1024 ? 2 : 1;
}

struct Cf {   // complex float with the same layout as HIP's float2
  float x, y;
};

// ------------------------------------------------------------ pass plan ---
constexpr int ilog2c(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Radix plans of a P-point transform. RM = 16 (default): the hand-picked
// plans below (2..16: one pass; 32..256: two; 512..4096: three). RM = 8 or 4:
// passes of at most 3 or 2 bits, larger passes first, for transforms whose
// radix-16 butterflies would leave threads idle (fewer points than 16 per
// thread): more passes, every thread busy.
constexpr int npass(int P, int RM = 16) {
  return RM >= 16 ? (P <= 16 ? 1 : (P <= 256 ? 2 : 3)) : (ilog2c(P) + ilog2c(RM) - 1) / ilog2c(RM);
}
constexpr int radix_of(int P, int s, int RM = 16) {
  return RM >= 16 ? (P <= 16 ? P
                     : P == 32 ? (s == 0 ? 8 : 4)
                     : P == 64 ? 8
                     : P == 128 ? (s == 0 ? 16 : 8)
                     : P == 256 ? 16
                     : P == 512 ? 8
                     : P == 1024 ? (s < 2 ? 16 : 4)
                     : P == 2048 ? (s < 2 ? 16 : 8)
                     : 16)
                  : 1 << (ilog2c(P) / npass(P, RM) + (s < ilog2c(P) % npass(P, RM) ? 1 : 0));
}

// Per-pass twiddle bases. A non-first pass with NS preceding points and radix
// R needs w^r = exp(DIR j 2 pi k r / (NS R)) for r = 1..R-1 at its butterfly
// index k. The table holds, per (plan, P, pass, k), the four bases w^1, w^2,
// w^4, w^8 (32 bytes, FP64-computed on the host); the other powers are
// products of at most three bases, so each butterfly loads two 16-byte
// vectors instead of R-1 separate twiddles, and all passes' bases are fetched
// when a transform starts, off the pass-to-pass critical path. Layout: the
// RM = 16 plans of all sizes, then the RM = 8 ones, then RM = 4.
constexpr int ns_of(int P, int s, int RM = 16) {
  int ns = 1;
  for (int t = 0; t < s; ++t) ns *= radix_of(P, t, RM);
  return ns;
}
constexpr int twb_size(int P, int s, int RM = 16) {
  return (s >= 1 && s < npass(P, RM)) ? 4 * ns_of(P, s, RM) : 0;
}
constexpr int twb_plan_total(int RM, int upto = 2 * kMaxPoints) {
  int off = 0;
  for (int q = 2; q < upto; q <<= 1)
    for (int t = 1; t < npass(q, RM); ++t) off += twb_size(q, t, RM);
  return off;
}
constexpr int twb_off(int P, int s, int RM = 16) {
  int off = (RM < 16 ? twb_plan_total(16) : 0) + (RM < 8 ? twb_plan_total(8) : 0) + twb_plan_total(RM, P);
  for (int t = 1; t < s; ++t) off += twb_size(P, t, RM);
  return off;
}
constexpr int twb_total() { return twb_plan_total(16) + twb_plan_total(8) + twb_plan_total(4); }
// largest radix for interleaved transforms of N points in all on 256 threads
constexpr int radix_cap(int N) { return N >= 4096 ? 16 : (N >= 2048 ? 8 : 4); }
// long FFT of the RX family under transform plan tp
constexpr int rx_long_cap(int N, int tp) { return tp && radix_cap(N) > 4 ? radix_cap(N) / 2 : radix_cap(N); }
constexpr bool rx_has_alt(int N) { return is_pow2c(N) && rx_long_cap(N, 1) != rx_long_cap(N, 0); }
// the same for one P-point transform on one wave (64 threads): radix 16 for
// 1024 points, 8 for 512, 4 below, so that from 256 points up every lane
// holds a butterfly in every pass (radix-16 passes left 48 of the 64 lanes
// idle at 256 points) and below it the fewest lanes idle that radix 4 allows
constexpr int wave_radix_cap(int P) { return P >= 1024 ? 16 : (P >= 512 ? 8 : 4); }

// One subband, shared by all operations.
struct SbDesc {
  int32_t L, logL;        // short transform length L_m
  int32_t c;              // centre bin c_m (signed)
  int32_t q0;             // (c_m - L_m/2) mod N: long bin of shifted index p = 0
  int32_t w_off;          // offset of this subband's weights in the weight table
  int32_t wave;           // RX: wave (0..3) running this subband's short IFFT, -1: whole workgroup
  int32_t cofs;           // RX: LDS offset (complex entries) of this subband's region
  int32_t aofs;           // weight gradient: offset (floats) of the subband's LDS accumulators;
                          // demodulating RX: complex offset of its terms in a task's slot
  int64_t lo_off;         // element offset of the subband's low-rate data for this op
  int64_t lo_len;         // number of low-rate samples for this op
};

// One processing group: subbands sharing a stream, n_long and a block grid.
struct GroupDesc {
  int32_t N, logN;
  int32_t n_sb, sb_first;    // subbands [sb_first, sb_first + n_sb) of the op's table
  int32_t prune;             // TX: 1 when the long IFFT is evaluated as N/L short IFFTs
  int32_t n_long_sb;         // RX: subbands whose short IFFT needs the whole workgroup (L > 1024)
  int32_t map_off;           // RX: offset of the group's scatter map (N entries) in LaunchArgs::rxmap
  int32_t scr_off;           // weight gradient: LDS offset (complex entries) of the short-FFT scratch
  int32_t wstride;           // weight gradient: scratch entries per wave (one-wave transforms)
  int32_t acc_off;           // weight gradient: LDS offset (complex entries) of the accumulators
  int32_t acc_len;           // weight gradient: accumulator floats (sum of the subbands' L);
                             // demodulating RX: complex values of a task's scratch slot
  int32_t taper;             // TX, synchronised OLS: edge length T of the output windows (0: hard edges)
  int32_t wg_nb;             // weight gradient, one subband with L <= 1024: blocks per group (0: per block)
  int32_t part_n;            // tasks of the group (scratch slots)
  int64_t part_base;         // first float of the group's scratch slots; the slot of the group's
                             // i-th task (block order) starts at part_base + i * (slot floats:
                             // acc_len for the weight gradient, 2 acc_len for the demodulating RX)
};

// One FC block of a group.
struct BlockDesc {
  int64_t t0;                // absolute high-rate element index of block sample 0
  int32_t hlo, hhi;          // TX: high-rate write window; RX: high-rate input window
  int32_t bs;                // index of the block's first BlockSb entry
  int32_t win;               // TX with taper: output window, see win_pack
};

// Output window of a tapered synchronised OLS TX block: support [lo, hi) of
// the block, a rising edge of T samples starting at lo and/or a falling edge
// of T samples ending at hi (T = GroupDesc::taper). lo, hi <= 4096.
constexpr int32_t win_pack(int lo, int hi, bool rise, bool fall) {
  return lo | (hi << 13) | ((rise ? 1 : 0) << 26) | ((fall ? 1 : 0) << 27);
}

// Per (block, subband).
struct BlockSb {
  int64_t x0;                // low-rate element index (absolute) of block sample 0;
                             // grid-input TX: first grid value of the block's symbol
  int32_t lo, hi;            // TX: valid input window; RX: low-rate keep window
  Cf ph;                     // TX: sqrt(I)/N * phi_r theta_n; RX: conj(phi_r theta_n)/(sqrt(I) L)
  int32_t shift;             // grid-input TX: block sample i is OFDM sample (i + shift) mod L
  int32_t K;                 // grid-input TX: active subcarriers of the subband
};

// A unit of work: a run of consecutive blocks of one group.
struct TaskDesc {
  int32_t group;
  int32_t blk_first, blk_count;
  int32_t warm;              // 1: the first block only feeds the OLA carry
  int64_t own_lo, own_hi;    // absolute high-rate (TX) / low-rate (RX) ownership
  int64_t z0_lo, z0_hi;      // zero-fill ranges inside the owned range (TX assign)
  int64_t z1_lo, z1_hi;
  int32_t ola;               // 1: blocks overlap-add their outputs (carry in LDS)
  int32_t accumulate;        // 1: out += value instead of out = value
  int64_t part_off;          // this task's scratch slot in LaunchArgs::part. Weight gradient:
                             // acc_len partial sums, in fftshifted weight order per subband at the
                             // subband's aofs; demodulating RX: the second block's terms, L complex
                             // values per subband at complex offset aofs
};

// Launch arguments of one kernel phase.
struct LaunchArgs {
  const SbDesc* sb;
  const GroupDesc* grp;
  const BlockDesc* blk;
  const BlockSb* bsb;
  const TaskDesc* task;
  int32_t n_task;
  int32_t io;
  const float* weights;
  const Cf* twiddle;         // exp(-j 2 pi k / kTwiddleN), k < kTwiddleN
  const Cf* twpass;          // per-pass twiddle bases (device code's twb_off layout)
  const uint64_t* rxmap;     // RX scatter maps: per long bin up to four 16-bit LDS destinations
  const void* in;
  void* out;
  const void* in2;           // weight gradient: the forward low-rate input
  int32_t front;             // TX: 1 = input is the QAM grid (OFDM modulation in the kernel)
  float* part;               // per-task scratch (weight gradient, demodulating RX)
  int32_t tplan;             // transform plan (0 or 1, see pruned_ws / rx_long_cap)
};

}  // namespace fcx

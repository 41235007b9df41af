// Device code of the fast-convolution (FC) filter banks for gfx950.
//
// One workgroup (256 threads, 4 wave64) processes one task: a run of
// consecutive FC blocks of one processing group.
// Transforms are Stockham FFTs held in LDS: every pass loads R values per
// butterfly into registers, applies the inter-pass twiddles (FP32 table built
// in FP64 on the host), runs a radix-R (2/4/8/16) DFT in registers and writes
// back in place after a barrier. Up to 16 complex values per thread, so one
// workgroup holds transforms of up to 4096 points (or batches of shorter ones
// with the same total), one wave up to 1024. Transform size, batch count and
// radix plan are compile-time, so all LDS offsets of a thread are one base
// register plus immediates. The first pass reads through a load functor
// (global memory or another LDS array) and the last pass hands its results
// to a store functor in registers, so segmentation, windowing, bin mapping,
// weighting and the overlap-add / overlap-save combination are fused into the
// transforms.
//
// Paper: Yli-Kaakinen et al., arXiv 2008.00672. TX follows the block operator
// W_N^{-1} M(phi) D P^(L/2) W_L A (Sec. III-B) and its symbol-synchronised
// form (Sec. III-C..III-E); RX follows W_L^{-1} P^(-L/2) D M^T W_N (Sec. IV).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "fc_internal.h"

namespace fcx {

// --------------------------------------------------------------- complex --
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by exp(DIR * j pi/2): DIR = -1 (forward) gives -j, DIR = +1 gives +j
template <int DIR>
__device__ __forceinline__ float2 mulj(float2 a) {
  return DIR < 0 ? make_float2(a.y, -a.x) : make_float2(-a.y, a.x);
}
template <int DIR>
__device__ __forceinline__ float2 cmulk(float2 a, float c, float s) {  // a * (c + DIR j s)
  return DIR < 0 ? make_float2(a.x * c + a.y * s, a.y * c - a.x * s)
                 : make_float2(a.x * c - a.y * s, a.y * c + a.x * s);
}

// ---------------------------------------------------- register DFTs ------
// X[k] = sum_n v[n] exp(DIR j 2 pi n k / R), in place, natural order.
template <int R, int DIR> struct Dft;

template <int DIR> struct Dft<2, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  }
};

template <int DIR>
__device__ __forceinline__ void dft4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = mulj<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR> struct Dft<4, DIR> {
  static __device__ __forceinline__ void run(float2* v) { dft4<DIR>(v[0], v[1], v[2], v[3]); }
};

template <int DIR> struct Dft<8, DIR> {
  static __device__ __forceinline__ void run(float2* v) {
    constexpr float h = 0.70710678118654752440f;
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    o1 = cmulk<DIR>(o1, h, h);                 // W8^1
    o2 = mulj<DIR>(o2);                        // W8^2
    o3 = cmulk<DIR>(o3, -h, h);                // W8^3
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  }
};

template <int DIR> struct Dft<16, DIR> {
  // 16 = 4 x 4: X[k1 + 4 k2] = sum_n2 W4^(n2 k2) W16^(n2 k1) sum_n1 v[n2 + 4 n1] W4^(n1 k1)
  static __device__ __forceinline__ void run(float2* v) {
    constexpr float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    constexpr float h = 0.70710678118654752440f;
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4<DIR>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
    // after the first layer, v[n2 + 4 k1] holds B[n2][k1]
    v[5] = cmulk<DIR>(v[5], c1, s1);           // n2=1,k1=1: W16^1
    v[9] = cmulk<DIR>(v[9], h, h);             // n2=1,k1=2: W16^2
    v[13] = cmulk<DIR>(v[13], s1, c1);         // n2=1,k1=3: W16^3
    v[6] = cmulk<DIR>(v[6], h, h);             // n2=2,k1=1: W16^2
    v[10] = mulj<DIR>(v[10]);                  // n2=2,k1=2: W16^4
    v[14] = cmulk<DIR>(v[14], -h, h);          // n2=2,k1=3: W16^6
    v[7] = cmulk<DIR>(v[7], s1, c1);           // n2=3,k1=1: W16^3
    v[11] = cmulk<DIR>(v[11], -h, h);          // n2=3,k1=2: W16^6
    v[15] = cmulk<DIR>(v[15], -c1, -s1);       // n2=3,k1=3: W16^9
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) dft4<DIR>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
    // now v[4 k1 + k2] holds X[k1 + 4 k2]: transpose to natural order
    float2 t[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = t[i];
  }
};

// v mod n for 0 <= v < 2n (any n: the mixed-radix sizes are not powers of two).
__device__ __forceinline__ int wrap(int v, int n) { return v >= n ? v - n : v; }

// LDS layout of the transform buffers between passes: one pad slot after
// every 32 elements, so the strided butterfly writes of the early passes
// spread over the banks. Buffers of n elements take lds_elems(n) slots.
__device__ __forceinline__ constexpr int pad(int e) { return e + (e >> 5); }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int NT>
__device__ __forceinline__ void group_sync() {
  if constexpr (NT == kThreads) __syncthreads(); else wave_sync();
}

// Twiddle bases of one butterfly: (w, w^2), and (w^4, w^8) for radix >= 8.
struct TwB {
  float4 v[2];
};

template <int P, int R, int LOGBT, int NT>
constexpr int maxit() { return (((P / R) << LOGBT) + NT - 1) / NT; }

template <int NT, int P, int LOGBT, int S, int RM, int MM>
__device__ __forceinline__ void twb_load(TwB (&t)[MM], const float2* __restrict__ twb, int tid) {
  constexpr int R = radix_of(P, S, RM);
  constexpr int NS = ns_of(P, S, RM);
  constexpr int TOTAL = (P / R) << LOGBT;
  constexpr int MAXIT = maxit<P, R, LOGBT, NT>();
  constexpr int OFF = twb_off(P, S, RM);      // folded here, not evaluated per call
  const float4* base = reinterpret_cast<const float4*>(twb + OFF);
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int g = tid + it * NT;
    if (TOTAL % NT == 0 || g < TOTAL) {
      const int k = (g >> LOGBT) & (NS - 1);
      t[it].v[0] = base[2 * k];
      if constexpr (R >= 8) t[it].v[1] = base[2 * k + 1];
    }
  }
}

template <int DIR>
__device__ __forceinline__ float2 twc(float a, float b) { return make_float2(a, DIR > 0 ? -b : b); }

// v[r] *= w^r for r = 1..R-1 (w^r from the four bases; DIR > 0 conjugates).
template <int R, int DIR>
__device__ __forceinline__ void apply_twiddles(float2* v, const TwB& t) {
  const float2 w1 = twc<DIR>(t.v[0].x, t.v[0].y);
  if constexpr (R == 2) {
    v[1] = cmul(v[1], w1);
  } else {
    const float2 w2 = twc<DIR>(t.v[0].z, t.v[0].w);
    const float2 w3 = cmul(w1, w2);
    v[1] = cmul(v[1], w1);
    v[2] = cmul(v[2], w2);
    v[3] = cmul(v[3], w3);
    if constexpr (R >= 8) {
      const float2 w4 = twc<DIR>(t.v[1].x, t.v[1].y);
      const float2 w5 = cmul(w1, w4), w6 = cmul(w2, w4), w7 = cmul(w3, w4);
      v[4] = cmul(v[4], w4);
      v[5] = cmul(v[5], w5);
      v[6] = cmul(v[6], w6);
      v[7] = cmul(v[7], w7);
      if constexpr (R == 16) {
        const float2 w8 = twc<DIR>(t.v[1].z, t.v[1].w);
        v[8] = cmul(v[8], w8);
        v[9] = cmul(v[9], cmul(w1, w8));
        v[10] = cmul(v[10], cmul(w2, w8));
        v[11] = cmul(v[11], cmul(w3, w8));
        v[12] = cmul(v[12], cmul(w4, w8));
        v[13] = cmul(v[13], cmul(w5, w8));
        v[14] = cmul(v[14], cmul(w6, w8));
        v[15] = cmul(v[15], cmul(w7, w8));
      }
    }
  }
}

// Mixed-radix transforms of P = 3 P2 points (is_tri(P)): three decimated
// P2-point sub-transforms, then a radix-3 combination (fft_run3). On one
// wave the sub-transforms run one after the other with the radix-4 plan
// (per thread S1 first-pass slots of each); on a workgroup waves 0..2 run
// one sub-transform each with the one-wave plan (per thread the P2 / 64
// first-pass slots of its wave's sub-transform). Per thread up to four
// output bins k2 of the combination (each giving three outputs).
constexpr int kTriRM = 4;
template <int NT, int P2>
constexpr int tri_s1() { return NT == kThreads ? P2 / 64 : (((P2 / 4) + NT - 1) / NT) * 4; }
template <int NT, int P2>
constexpr int tri_j() { return (P2 + NT - 1) / NT; }

template <int NT, int P, int LOGBT, int RM = 16>
__device__ __forceinline__ bool first_pos(int s, int tid, int& i, int& b);

// Slot s of the first pass: element index i and transform b it loads.
// (Mixed radix: slot n1 S1 + s' is first-pass slot s' of sub-transform n1,
// element i = 3 i2 + n1.)
template <int NT, int P, int LOGBT, int RM>
__device__ __forceinline__ bool first_pos(int s, int tid, int& i, int& b) {
  if constexpr (is_tri(P)) {
    static_assert(LOGBT == 0, "mixed-radix transforms are not interleaved");
    constexpr int P2 = P / 3, S1 = tri_s1<NT, P2>();
    int n1, i2;
    if constexpr (NT == kThreads) {          // wave n1 holds sub-transform n1
      n1 = tid >> 6;
      if (n1 >= 3 || !first_pos<64, P2, 0, wave_radix_cap(P2)>(s, tid & 63, i2, b)) return false;
    } else {
      n1 = s / S1;
      if (n1 >= 3 || !first_pos<NT, P2, 0, kTriRM>(s - n1 * S1, tid, i2, b)) return false;
    }
    i = 3 * i2 + n1;
    return true;
  }
  constexpr int R = radix_of(P, 0, RM);
  constexpr int NB = P / R;
  constexpr int TOTAL = NB << LOGBT;
  const int it = s / R, r = s % R;
  const int g = tid + it * NT;
  if (g >= TOTAL) return false;
  b = g & ((1 << LOGBT) - 1);
  i = (g >> LOGBT) + r * NB;
  return true;
}

// Output position of register slot s of the last pass (-1: slot unused).
// (Mixed radix: slot 3 j + k1 is output k2 + P2 k1, k2 = tid + j NT.)
template <int NT, int P, int LOGBT, int RM = 16>
__device__ __forceinline__ int last_pos(int s, int tid) {
  if constexpr (is_tri(P)) {
    constexpr int P2 = P / 3;
    const int j = s / 3, k2 = tid + j * NT;
    if (j >= tri_j<NT, P2>() || k2 >= P2) return -1;
    return k2 + P2 * (s - 3 * j);
  }
  constexpr int R = radix_of(P, npass(P, RM) - 1, RM);
  constexpr int NB = P / R;
  constexpr int TOTAL = NB << LOGBT;
  const int it = s / R, r = s % R;
  const int g = tid + it * NT;
  if (g >= TOTAL) return -1;
  const int b = g & ((1 << LOGBT) - 1), j = g >> LOGBT;
  return ((j + r * NB) << LOGBT) + b;
}

// One Stockham pass over P-point transforms, 2^LOGBT of them interleaved
// (element i of transform b at index i * 2^LOGBT + b), run by NT threads.
// NS is the product of the radices of the previous passes. The first pass
// reads through load(slot, i, b, ip); the last hands results to
// store(slot, t, v, tp); ip / tp are the padded LDS positions of the element.
template <int NT, int P, int LOGBT, int R, int NS, int DIR, bool FIRST, bool LAST, class Load, class Store>
__device__ __forceinline__ void fft_pass(float2* __restrict__ buf, int tid, Load& load, Store& store,
                                         const TwB* tb) {
  constexpr int NB = P / R;
  constexpr int BT = 1 << LOGBT;
  constexpr int TOTAL = NB * BT;
  constexpr int MAXIT = (TOTAL + NT - 1) / NT;
  static_assert(MAXIT * R <= 16, "at most 16 complex values per thread");
  float2 v[MAXIT][R];
  // LDS offsets: element base + r * S sits at pad(base) + r * S + (r * S) / 32
  // for every thread (base < S when S < 32; S a multiple of 32 otherwise), so
  // each access is one per-thread base plus a compile-time offset.
  constexpr int SR = NB * BT;            // read stride
  constexpr int SW = NS * BT;            // write stride
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int g = tid + it * NT;
    if (TOTAL % NT == 0 || g < TOTAL) {
      const int b = g & (BT - 1), j = g >> LOGBT;
      if constexpr (FIRST) {
        const int p0 = pad((j << LOGBT) + b);
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = load(it * R + r, j + r * NB, b, p0 + r * SR + ((r * SR) >> 5));
      } else {
        const float2* rp = buf + pad((j << LOGBT) + b);
#pragma unroll
        for (int r = 0; r < R; ++r) v[it][r] = rp[r * SR + ((r * SR) >> 5)];
      }
    }
  }
  group_sync<NT>();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int g = tid + it * NT;
    if (TOTAL % NT == 0 || g < TOTAL) {
      const int b = g & (BT - 1), j = g >> LOGBT;
      const int k = j & (NS - 1);
      if constexpr (!FIRST) apply_twiddles<R, DIR>(v[it], tb[it]);
      Dft<R, DIR>::run(v[it]);
      if constexpr (LAST) {
        const int p0 = pad((j << LOGBT) + b);
#pragma unroll
        for (int r = 0; r < R; ++r)
          store(it * R + r, ((j + r * NB) << LOGBT) + b, v[it][r], p0 + r * SR + ((r * SR) >> 5));
      } else {
        float2* wp = buf + pad((((j - k) * R + k) << LOGBT) + b);
#pragma unroll
        for (int r = 0; r < R; ++r) wp[r * SW + ((r * SW) >> 5)] = v[it][r];
      }
    }
  }
  if constexpr (!LAST) group_sync<NT>();
}

// Largest number of per-thread transform slots over the non-first passes.
template <int NT, int P, int LOGBT, int RM>
constexpr int max_maxit() {
  int m = 1;
  for (int s = 1; s < npass(P, RM); ++s) {
    const int R = radix_of(P, s, RM);
    const int v = (((P / R) << LOGBT) + NT - 1) / NT;
    if (v > m) m = v;
  }
  return m;
}

template <int NT, int P, int LOGBT, int RM, int S, int MM>
__device__ __forceinline__ void twb_load_from(TwB (*t)[MM], const float2* __restrict__ twb, int tid) {
  if constexpr (S < npass(P, RM)) {
    twb_load<NT, P, LOGBT, S, RM, MM>(t[S - 1], twb, tid);
    twb_load_from<NT, P, LOGBT, RM, S + 1, MM>(t, twb, tid);
  }
}

template <int NT, int P, int LOGBT, int DIR, int RM, int S, int MM, class Load, class Store>
__device__ __forceinline__ void passes_from(float2* buf, int tid, Load& load, Store& store, TwB (*t)[MM]) {
  constexpr int NP = npass(P, RM);
  fft_pass<NT, P, LOGBT, radix_of(P, S, RM), ns_of(P, S, RM), DIR, S == 0, S == NP - 1>(
      buf, tid, load, store, t[S == 0 ? 0 : S - 1]);
  if constexpr (S + 1 < NP) passes_from<NT, P, LOGBT, DIR, RM, S + 1, MM>(buf, tid, load, store, t);
}

// Whole transform: DIR = -1 forward DFT, +1 unnormalised inverse, of 2^LOGBT
// interleaved P-point transforms with the radix plan RM (see radix_of). The
// caller provides a barrier before the call when `buf`, or what `load`
// reads, was written by other threads. load.prefetch / store.prefetch are
// called first, so functors can start their own global loads (weights,
// twiddles) before the passes run; every pass's twiddle bases are fetched
// then as well.
template <int NT, int P, int DIR, class Load, class Store>
__device__ __forceinline__ void fft_run3(float2* buf, int tid, Load& load, Store& store, const float2* twb);

template <int NT, int P, int LOGBT, int DIR, int RM = 16, class Load, class Store>
__device__ __forceinline__ void fft_run(float2* buf, int tid, Load& load, Store& store,
                                        const float2* __restrict__ twb) {
  if constexpr (is_tri(P)) {
    static_assert(LOGBT == 0, "mixed-radix transforms are not interleaved");
    fft_run3<NT, P, DIR>(buf, tid, load, store, twb);
    return;
  } else {
  constexpr int NP = npass(P, RM);
  static_assert(NT == kThreads || P <= 1024, "one wave holds at most 1024 points");
  // All LDS and twiddle indices of a pass depend only on the thread, so the
  // compiler would compute every transform's indices (and twiddle loads) once
  // outside the block loops and keep them all live for the whole kernel. That
  // costs far more occupancy than recomputing them costs ALU, so both the
  // thread index and the table pointer are made opaque per transform.
  asm volatile("" : "+v"(tid));
  asm volatile("" : "+s"(twb));
  constexpr int MM = max_maxit<NT, P, LOGBT, RM>();
  TwB t[NP > 1 ? NP - 1 : 1][MM];
  twb_load_from<NT, P, LOGBT, RM, 1, MM>(t, twb, tid);
  load.prefetch(tid);
  store.prefetch(tid);
  passes_from<NT, P, LOGBT, DIR, RM, 0, MM>(buf, tid, load, store, t);
  }
}

template <int V> struct SizeC { static constexpr int value = V; };

// Functors without prefetch work derive from this.
struct NoPrefetch {
  __device__ __forceinline__ void prefetch(int) {}
};

// Uses a functor whose prefetch already ran (fft_run's prefetch call is a no-op).
template <class F> struct NoPrefetchWrap {
  F& f;
  __device__ __forceinline__ void prefetch(int) {}
  template <class... A>
  __device__ __forceinline__ auto operator()(A... args) -> decltype(f(args...)) { return f(args...); }
};

// First pass of a sub-transform of fft_run3: its inputs, loaded before any
// sub-transform wrote the buffer.
template <int S1> struct LoadRegs : NoPrefetch {
  const float2* x;
  __device__ __forceinline__ float2 operator()(int slot, int, int, int) const { return x[slot]; }
};

// Last pass of a sub-transform of fft_run3: bin k2 at its padded position.
struct StoreRegion : NoPrefetch {
  float2* buf;
  __device__ __forceinline__ void operator()(int, int, float2 v, int tp) const { buf[tp] = v; }
};

// P = 3 P2 points (Cooley-Tukey with the factor 3 first: n = 3 n2 + n1,
// k = k2 + P2 k1):
//   T_n1[k2] = sum_n2 x[3 n2 + n1] W_P2^(n2 k2)          (three P2-point DFTs)
//   X[k2 + P2 k1] = sum_n1 (W_P^(n1 k2) T_n1[k2]) W_3^(n1 k1)
// with W_n = exp(DIR j 2 pi / n). Every input goes to registers first (the
// buffer may hold the input), then sub-transform n1 runs in the n1-th third
// of the buffer (pad(k2 + P2 k1) = k1 lds_elems(P2) + pad(k2), since P2 is a
// multiple of 32), and the combination reads the three values of its bins
// into registers before the outputs are stored (a store functor may write
// anywhere in the buffer). Same functor contract as fft_run.
template <int NT, int P, int DIR, class Load, class Store>
__device__ __forceinline__ void fft_run3(float2* buf, int tid, Load& load, Store& store, const float2* twb) {
  constexpr int P2 = P / 3, S1 = tri_s1<NT, P2>(), J = tri_j<NT, P2>(), LE = lds_elems(P2);
  constexpr bool kWaves = NT == kThreads;           // one sub-transform per wave
  constexpr int NSUB = kWaves ? 1 : 3;               // sub-transforms loaded by each thread
  static_assert(NSUB * S1 <= 16 && 3 * J <= 16, "at most 16 values per thread");
  static_assert(P2 % 32 == 0, "sub-transforms align with the LDS padding");
  asm volatile("" : "+v"(tid));
  load.prefetch(tid);
  store.prefetch(tid);
  float2 x[NSUB][S1];
#pragma unroll
  for (int n1 = 0; n1 < NSUB; ++n1)
#pragma unroll
    for (int q = 0; q < S1; ++q) {
      int i, b;
      if (first_pos<NT, P, 0>(n1 * S1 + q, tid, i, b)) x[n1][q] = load(n1 * S1 + q, i, b, pad(i));
    }
  group_sync<NT>();
  if constexpr (kWaves) {
    const int w = tid >> 6;
    if (w < 3) {
      LoadRegs<S1> lr;
      lr.x = x[0];
      StoreRegion sr;
      sr.buf = buf + w * LE;
      fft_run<64, P2, 0, DIR, wave_radix_cap(P2)>(buf + w * LE, tid & 63, lr, sr, twb);
    }
  } else {
#pragma unroll
    for (int n1 = 0; n1 < 3; ++n1) {
      LoadRegs<S1> lr;
      lr.x = x[n1];
      StoreRegion sr;
      sr.buf = buf + n1 * LE;
      fft_run<NT, P2, 0, DIR, kTriRM>(buf + n1 * LE, tid, lr, sr, twb);
    }
  }
  group_sync<NT>();
  constexpr int kTw3Off = twb_total();                // folded here, not evaluated per call
  const float2* tw3 = twb + kTw3Off;
  float2 v[J][3];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k2 = tid + j * NT;
    if (P2 % NT == 0 || k2 < P2) {
      const int p = pad(k2);
      v[j][0] = buf[p];
      v[j][1] = buf[LE + p];
      v[j][2] = buf[2 * LE + p];
    }
  }
  group_sync<NT>();
  constexpr float h3 = 0.86602540378443864676f;       // sin(2 pi / 3)
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int k2 = tid + j * NT;
    if (P2 % NT == 0 || k2 < P2) {
      const float2 w1 = tw3[k2 * (kTw3N / P)], w2 = tw3[2 * k2 * (kTw3N / P)];
      const float2 a = v[j][0];
      const float2 b = cmul(v[j][1], make_float2(w1.x, DIR > 0 ? -w1.y : w1.y));
      const float2 c = cmul(v[j][2], make_float2(w2.x, DIR > 0 ? -w2.y : w2.y));
      // W_3 = -1/2 + DIR j sin(2 pi/3): X1 = m + d, X2 = m - d
      const float2 sbc = cadd(b, c);
      const float2 m = make_float2(a.x - 0.5f * sbc.x, a.y - 0.5f * sbc.y);
      const float2 d = cscale(mulj<DIR>(csub(b, c)), h3);
      store(3 * j, k2, cadd(a, sbc), pad(k2));
      store(3 * j + 1, k2 + P2, cadd(m, d), LE + pad(k2));
      store(3 * j + 2, k2 + 2 * P2, csub(m, d), 2 * LE + pad(k2));
    }
  }
}

// ------------------------------------------------------------------- I/O --
// Interleaved I/Q storage; element pointers are formed once per block from the
// uniform 64-bit offsets, per-sample indices are 32-bit.
template <int IO> struct Io;
template <> struct Io<IO_C64> {
  using T = float2;
  static __device__ __forceinline__ float2 ld(const T* p, int i) { return p[i]; }
  static __device__ __forceinline__ void st(T* p, int i, float2 v) { p[i] = v; }
};
template <> struct Io<IO_F16> {
  using T = __half2;
  static __device__ __forceinline__ float2 ld(const T* p, int i) { return __half22float2(p[i]); }
  static __device__ __forceinline__ void st(T* p, int i, float2 v) { p[i] = __float22half2_rn(v); }
};
// gfx950 converts a float pair to bfloat16 with round-to-nearest-even in one
// instruction (v_cvt_pk_bf16_f32), which the __bf16 conversions select.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
template <> struct Io<IO_BF16> {
  using T = uint32_t;
  static __device__ __forceinline__ float2 ld(const T* p, int i) {
    const uint32_t u = p[i];
    return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
  }
  static __device__ __forceinline__ void st(T* p, int i, float2 v) {
    bf16x2_t r;
    r.x = (__bf16)v.x;
    r.y = (__bf16)v.y;
    p[i] = __builtin_bit_cast(uint32_t, r);
  }
};

template <int IO>
__device__ __forceinline__ const typename Io<IO>::T* at(const void* p, int64_t off) {
  return reinterpret_cast<const typename Io<IO>::T*>(p) + off;
}
template <int IO>
__device__ __forceinline__ typename Io<IO>::T* at(void* p, int64_t off) {
  return reinterpret_cast<typename Io<IO>::T*>(p) + off;
}
template <int IO>
__device__ __forceinline__ void put(typename Io<IO>::T* p, int i, float2 v, bool acc) {
  if (acc) v = cadd(v, Io<IO>::ld(p, i));
  Io<IO>::st(p, i, v);
}

// ------------------------------------------------------------- functors ---
// Low-rate segment: block sample i is x[i] inside [lo, hi), else 0.
template <int IO> struct LoadSeg : NoPrefetch {
  const typename Io<IO>::T* x; int lo, hi;
  __device__ __forceinline__ float2 operator()(int, int i, int, int) const {
    return (i >= lo && i < hi) ? Io<IO>::ld(x, i) : make_float2(0.f, 0.f);
  }
};

// Input segment whose first-pass samples were loaded ahead of time (raw
// storage words in registers): issue() starts the loads, typically while the
// previous block is still being transformed; operator() converts on use.
template <int IO, int NT, int P, int RM = 16> struct LoadAhead : NoPrefetch {
  using T = typename Io<IO>::T;
  T raw[16];
  unsigned valid;
  __device__ __forceinline__ void issue(const T* x, int lo, int hi, int tid) { issue_sized<P, RM>(x, lo, hi, tid); }
  // The same for a PP-point transform with radix plan RMM (the slots' layout
  // does not depend on them, so one object can serve transforms of a size
  // known at run time).
  template <int PP, int RMM = 16>
  __device__ __forceinline__ void issue_sized(const T* x, int lo, int hi, int tid) {
    // keep the loads where they are issued: hoisted above the transform that
    // precedes them they would only lengthen register live ranges
    asm volatile("" : "+v"(tid) : : "memory");
    valid = 0;
    if (lo <= 0 && hi >= PP) {
      // the whole block is valid (a uniform branch): no per-sample checks
#pragma unroll
      for (int s = 0; s < 16; ++s) {
        int i, b;
        if (first_pos<NT, PP, 0, RMM>(s, tid, i, b)) {
          raw[s] = x[i];
          valid |= 1u << s;
        }
      }
      return;
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int i, b;
      if (first_pos<NT, PP, 0, RMM>(s, tid, i, b) && i >= lo && i < hi) {
        raw[s] = x[i];
        valid |= 1u << s;
      }
    }
  }
  // The first pass of an L-point IFFT of one QAM symbol: bin i carries grid
  // value kappa + K/2 for kappa = i (i < K/2) or i - P (i >= P - K/2), else 0.
  __device__ __forceinline__ void issue_grid(const T* row, int K, int tid) {
    asm volatile("" : "+v"(tid) : : "memory");
    valid = 0;
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int i, b;
      if (first_pos<NT, P, 0, RM>(s, tid, i, b)) {
        const int g = i < (K >> 1) ? i + (K >> 1) : (i >= P - (K >> 1) ? i - P + (K >> 1) : -1);
        if (g >= 0) {
          raw[s] = row[g];
          valid |= 1u << s;
        }
      }
    }
  }
  __device__ __forceinline__ float2 operator()(int slot, int, int, int) const {
    return (valid >> slot) & 1u ? Io<IO>::ld(raw, slot) : make_float2(0.f, 0.f);
  }
};

// The same mapping without prefetch (one grid row of an L-point symbol).
template <int IO, int L> struct LoadGridRow : NoPrefetch {
  const typename Io<IO>::T* row; int K;
  __device__ __forceinline__ float2 operator()(int, int i, int, int) const {
    const int g = i < (K >> 1) ? i + (K >> 1) : (i >= L - (K >> 1) ? i - L + (K >> 1) : -1);
    return g >= 0 ? Io<IO>::ld(row, g) : make_float2(0.f, 0.f);
  }
};

// Last pass of the OFDM IFFT: x[t] = IFFT(X)[t] / sqrt(L), natural order.
struct StoreScaled : NoPrefetch {
  float2* buf; float scale;
  __device__ __forceinline__ void operator()(int, int, float2 v, int tp) const {
    buf[tp] = make_float2(v.x * scale, v.y * scale);
  }
};

// First pass of the FC short FFT of a symbol-synchronised block taken from the
// OFDM symbol in LDS: block sample i in the window [lo, hi) is OFDM sample
// (i + shift) mod L (the CP and the zero padding are index ranges).
template <int L> struct LoadCyclic : NoPrefetch {
  const float2* x; int lo, hi, shift;
  __device__ __forceinline__ float2 operator()(int, int i, int, int) const {
    return (i >= lo && i < hi) ? x[pad(wrap(i + shift, L))] : make_float2(0.f, 0.f);
  }
};

// Natural-order LDS read (first pass reading an LDS spectrum).
struct LoadLds : NoPrefetch {
  const float2* s;
  __device__ __forceinline__ float2 operator()(int, int i, int, int) const { return s[i]; }
};

// TX, pruned long IFFT: short-FFT bin u -> residue rho = (u + c) mod L of the
// band, weighted by D[p] (p = (u + L/2) mod L, the fftshifted index) and the
// block phase. The weights of this thread's output bins are fetched when the
// transform starts.
template <int NT, int L, int RM = 16> struct StoreBand {
  static_assert(is_pow2c(L), "the pruned long IFFT takes power-of-two sizes");
  float2* V; const float* D; float2 ph; int c;
  float d[16];
  __device__ __forceinline__ void prefetch(int tid) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int u = last_pos<NT, L, 0, RM>(s, tid);
      if (u >= 0) d[s] = D[(u + (L >> 1)) & (L - 1)];
    }
  }
  __device__ __forceinline__ void operator()(int slot, int u, float2 v, int) const {
    V[(u + c) & (L - 1)] = cscale(cmul(v, ph), d[slot]);
  }
};

// TX, pruned long IFFT first pass: sub-transform b (output samples t = a*I + b)
// of residue rho takes V[rho] * exp(+j 2 pi q b / N), q the band bin of rho.
// The twiddles depend only on the thread and the subband, so they are fetched
// before the short FFT of the block runs.
template <int NT, int L, int LOGI, int RM> struct LoadPruned {
  static constexpr int N = L << LOGI;
  const float2* V; const float2* tw; int q0;
  float2 w[16];
  __device__ __forceinline__ void prefetch(int tid) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int rho, b;
      if (first_pos<NT, L, LOGI, RM>(s, tid, rho, b)) {
        const int q = (q0 + ((rho - q0) & (L - 1))) & (N - 1);
        w[s] = tw[((q * b) & (N - 1)) * (kTwiddleN / N)];
      }
    }
  }
  __device__ __forceinline__ float2 operator()(int slot, int rho, int, int) const {
    return cmul(V[rho], make_float2(w[slot].x, -w[slot].y));
  }
};

// TX, full long IFFT: add the weighted band into the N-bin spectrum.
template <int N> struct StoreAddLong : NoPrefetch {
  float2* S; const float* D; float2 ph; int L, q0;
  __device__ __forceinline__ void operator()(int, int u, float2 v, int) const {
    const int p = wrap(u + (L >> 1), L);
    const int q = wrap(q0 + p, N);
    S[q] = cadd(S[q], cscale(cmul(v, ph), D[p]));
  }
};

// TX epilogue, phase 1 (inside the last pass): OLA carry-in for block samples
// t < pth; results stay in registers until phase 2.
struct TxEpi : NoPrefetch {
  const float2* pend; int pth;
  float2 val[16];
  __device__ __forceinline__ void operator()(int slot, int t, float2 v, int) {
    if (t < pth) v = cadd(v, pend[t]);
    val[slot] = v;
  }
};

// Same, with the output window of a tapered synchronised OLS block applied
// before the carry-in (taper = 0: no window). The window is zero outside
// [lo, hi), one inside, with a rising edge w_i = sin^2(pi (i + 1/2) / (2T))
// over [lo, lo + T) and/or the mirrored falling edge over [hi - T, hi).
struct TxEpiWin : TxEpi {
  int lo, hi, taper; bool rise, fall;
  __device__ __forceinline__ void set_window(int32_t win, int T) {
    lo = win & 8191; hi = (win >> 13) & 8191; rise = (win >> 26) & 1; fall = (win >> 27) & 1; taper = T;
  }
  __device__ __forceinline__ float ramp(int i) const {
    const float s = sinf(3.14159265358979f * (float)(2 * i + 1) / (float)(4 * taper));
    return s * s;
  }
  __device__ __forceinline__ void operator()(int slot, int t, float2 v, int tp) {
    if (taper) {
      float w = (t >= lo && t < hi) ? 1.f : 0.f;
      if (rise && t >= lo && t < lo + taper) w = ramp(t - lo);
      if (fall && t >= hi - taper && t < hi) w = ramp(hi - 1 - t);
      v = cscale(v, w);
    }
    TxEpi::operator()(slot, t, v, tp);
  }
};

// RX, last pass of the long FFT: each bin q goes straight to every subband
// region that gathers it (up to four LDS destinations per bin, 16 bits each,
// 0xffff = none; built by the planner). The regions overlay the spectrum: all
// reads of the last pass finished at its barrier. The destinations are read
// (from cache) only when the bins are stored: holding them through the
// transform would cost 32 registers per thread and one wave per SIMD.
struct StoreScatter : NoPrefetch {
  float2* S; const uint64_t* map;
  __device__ __forceinline__ void operator()(int, int t, float2 v, int) const {
    const uint64_t e = map[t];
    const uint32_t e01 = (uint32_t)e, e23 = (uint32_t)(e >> 32);
    if ((e01 & 0xffffu) != 0xffffu) S[e01 & 0xffffu] = v;
    if ((e01 >> 16) != 0xffffu) S[e01 >> 16] = v;
    if (e23 != 0xffffffffu) {          // third and fourth destinations are rare
      if ((e23 & 0xffffu) != 0xffffu) S[e23 & 0xffffu] = v;
      if ((e23 >> 16) != 0xffffu) S[e23 >> 16] = v;
    }
  }
};


// High-rate segment with an input window [lo, hi).
template <int IO> struct LoadHigh : NoPrefetch {
  const typename Io<IO>::T* x; int lo, hi;
  __device__ __forceinline__ float2 operator()(int, int i, int, int) const {
    return (i >= lo && i < hi) ? Io<IO>::ld(x, i) : make_float2(0.f, 0.f);
  }
};


// RX short IFFT first pass from the subband's compacted region (bin u of the
// subband at region[pad(u)], already in inverse-shift order), weighted by
// D[p]; the transform then runs in place in the region. The block's conj
// phase, one complex factor per block and subband, multiplies the kept
// outputs instead (StoreLow: half of the L values for overlap 1/2).
// The weights of this thread's first-pass bins are fetched when the transform
// starts, together with its twiddle bases (their registers live only until
// the first pass: the RX kernel keeps four waves per SIMD; 2 % off the RX
// call against reading them at use).
template <int NT, int L> struct LoadCompact {
  const float2* R; const float* D;
  float d[16];
  __device__ __forceinline__ void prefetch(int tid) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int u, b;
      if (first_pos<NT, L, 0, NT == 64 ? wave_radix_cap(L) : radix_cap(L)>(s, tid, u, b))
        d[s] = D[wrap(u + (L >> 1), L)];
    }
  }
  __device__ __forceinline__ float2 operator()(int slot, int, int, int up) const {
    return cscale(R[up], d[slot]);
  }
};

// RX output: keep window [lo, hi) of the low-rate block, times the block's
// conj phase.
template <int IO> struct StoreLow : NoPrefetch {
  typename Io<IO>::T* out; int lo, hi; bool acc; float2 ph;
  __device__ __forceinline__ void operator()(int, int i, float2 v, int) const {
    if (i >= lo && i < hi) put<IO>(out, i, cmul(v, ph), acc);
  }
};

// ------------------------------------------------------------- TX tasks ---
// Block-local 32-bit view of the OLA/OLS bookkeeping of one TX block.
struct TxWin {
  int pth;    // samples t < pth add the carry of the previous block
  int cth;    // samples t >= cth go to the carry of the next block
  int wlo, whi;   // samples written to the output
};

__device__ __forceinline__ TxWin tx_window(const BlockDesc& B, const TaskDesc& T, int64_t prev_end,
                                           int64_t next_start, int n) {
  TxWin w;
  w.pth = prev_end > B.t0 ? (int)(prev_end - B.t0) : 0;
  w.cth = next_start < B.t0 + n ? (int)(next_start - B.t0) : n;
  int64_t lo = T.own_lo - B.t0, hi = T.own_hi - B.t0;
  lo = lo > B.hlo ? lo : B.hlo;
  hi = hi < B.hhi ? hi : B.hhi;
  if (hi < lo) hi = lo;
  w.wlo = (int)(lo < 0 ? 0 : (lo > n ? n : lo));
  w.whi = (int)(hi < 0 ? 0 : (hi > n ? n : hi));
  return w;
}

// Epilogue phase 2 (after a barrier): OLA carry-out or write the owned samples.
template <int IO, int NT, int P, int LOGBT, int RM = 16>
__device__ __forceinline__ void tx_epilogue(const TxEpi& ep, float2* pend, const TxWin& w,
                                            typename Io<IO>::T* ob, bool acc, int tid) {
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = last_pos<NT, P, LOGBT, RM>(s, tid);
    if (t < 0) continue;
    if (t >= w.cth) pend[t - w.cth] = ep.val[s];
    else if (t >= w.wlo && t < w.whi) put<IO>(ob, t, ep.val[s], acc);
  }
}

template <int IO>
__device__ __forceinline__ void zero_span(void* out, int64_t lo, int64_t hi) {
  if (hi <= lo) return;
  typename Io<IO>::T* p = at<IO>(out, lo);
  const int n = (int)(hi - lo);
  for (int i = threadIdx.x; i < n; i += kThreads) Io<IO>::st(p, i, make_float2(0.f, 0.f));
}

// Single-subband group, N = L * 2^LOGI: short FFT, then the long IFFT
// evaluated as 2^LOGI interleaved L-point IFFTs of the twiddled band (outputs
// land in natural order). Where pruned_wave_short(L, N) holds, the blocks go
// in groups of up to four: each wave runs the short FFT of one block of the
// group into its own band region, then the workgroup runs the group's long
// IFFTs and epilogues in block order (the OLA carry passes from block to
// block through LDS). Otherwise one block at a time, the short FFT on the
// whole workgroup in the long IFFT buffer.
template <int IO, int L, int LOGI, bool FRONT, int TP>
__global__ __launch_bounds__(kThreads, pruned_waves_per_simd(L, L << LOGI, TP)) void fc_tx_pruned_kernel(LaunchArgs a) {
  constexpr int N = L << LOGI;
  constexpr bool kWaveShort = pruned_ws(L, N, TP);          // transform plan TP
  constexpr int NB = pruned_group_blocks(L, N, TP);         // blocks per group
  // the long IFFT's first-pass twiddles depend only on the thread and the
  // subband: fetched once per task and kept in registers where the LDS
  // already limits occupancy to two workgroups per CU (registers are free)
  constexpr bool kKeepTwiddles = N <= 2048 && pruned_waves_per_simd(L, N, TP) <= 2;
  extern __shared__ float2 smem[];
  const int task = blockIdx.x;
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  if (!T.accumulate) {
    zero_span<IO>(a.out, T.z0_lo, T.z0_hi);
    zero_span<IO>(a.out, T.z1_lo, T.z1_hi);
  }
  const SbDesc S = a.sb[G.sb_first];
  float2* buf = smem;                         // long IFFT (and, not kWaveShort, short FFT and band)
  float2* pend = smem + lds_elems(N);         // OLA carry, up to N/2 points
  float2* bands = pend + N / 2;               // kWaveShort: one short-FFT / band region per wave
  const float* D = a.weights + S.w_off;
  const float2* tw = reinterpret_cast<const float2*>(a.twiddle);
  const float2* twb = reinterpret_cast<const float2*>(a.twpass);
  const int tid = threadIdx.x;
  const int wave = kWaveShort ? tid >> 6 : 0;             // waves >= NB idle in the short phase
  // for N <= 512 even radix-4 passes keep only N/4 threads busy: rotating
  // the thread roles with the workgroup index spreads those threads' waves
  // over the CU's SIMDs instead of loading the first SIMD(s) in every
  // workgroup
  const int rtid = (tid + 64 * (int)(blockIdx.x & 3)) & (kThreads - 1);
  const int sid = kWaveShort ? tid & 63 : tid;          // index within the short FFT's threads
  constexpr int NTS = kWaveShort ? 64 : kThreads;
  constexpr int RMS = kWaveShort ? wave_radix_cap(L) : radix_cap(L);   // short-FFT radix plan
  float2* band = kWaveShort ? bands + wave * lds_elems(L) : buf;
  int64_t prev_end = INT64_MIN;
  LoadAhead<IO, NTS, L, RMS> ld;
  if (wave < NB && wave < T.blk_count) {
    const BlockSb Z0 = a.bsb[a.blk[T.blk_first + wave].bs];
    if constexpr (FRONT) ld.issue_grid(at<IO>(a.in, Z0.x0), Z0.K, sid);
    else ld.issue(at<IO>(a.in, Z0.x0), Z0.lo, Z0.hi, sid);
  }
  // radix plan of the long IFFT: every thread takes part in every pass
  constexpr int RM = radix_cap(N);
  LoadPruned<kThreads, L, LOGI, RM> lp;
  lp.tw = tw; lp.q0 = S.q0;
  if constexpr (kKeepTwiddles) lp.prefetch(rtid);
  for (int g0 = 0; g0 < T.blk_count; g0 += NB) {
    const int nb = T.blk_count - g0 < NB ? T.blk_count - g0 : NB;
    __syncthreads();
    if (wave < nb) {
      const BlockSb Zw = a.bsb[a.blk[T.blk_first + g0 + wave].bs];
      StoreBand<NTS, L, RMS> sb;
      sb.V = band; sb.D = D; sb.ph = make_float2(Zw.ph.x, Zw.ph.y); sb.c = S.c;
      if constexpr (FRONT) {
        // grid input: the symbol's OFDM IFFT in the band region, then the
        // block's short FFT from it
        StoreScaled sx;
        sx.buf = band; sx.scale = rsqrtf((float)L);
        fft_run<NTS, L, 0, +1, RMS>(band, sid, ld, sx, twb);
        group_sync<NTS>();
        LoadCyclic<L> lcy;
        lcy.x = band; lcy.lo = Zw.lo; lcy.hi = Zw.hi; lcy.shift = Zw.shift;
        fft_run<NTS, L, 0, -1, RMS>(band, sid, lcy, sb, twb);
      } else {
        fft_run<NTS, L, 0, -1, RMS>(band, sid, ld, sb, twb);
      }
    }
    // start loading the next group's inputs while this group's IFFTs run
    if (wave < NB && g0 + NB + wave < T.blk_count) {
      const BlockSb Zn = a.bsb[a.blk[T.blk_first + g0 + NB + wave].bs];
      if constexpr (FRONT) ld.issue_grid(at<IO>(a.in, Zn.x0), Zn.K, sid);
      else ld.issue(at<IO>(a.in, Zn.x0), Zn.lo, Zn.hi, sid);
    }
    for (int k = 0; k < nb; ++k) {
      const int bi = g0 + k;
      const BlockDesc B = a.blk[T.blk_first + bi];
      const int64_t next_start =
          (T.ola && bi + 1 < T.blk_count) ? a.blk[T.blk_first + bi + 1].t0 : INT64_MAX;
      const TxWin w = tx_window(B, T, prev_end, next_start, N);
      lp.V = kWaveShort ? bands + k * lds_elems(L) : buf;
      __syncthreads();
      TxEpi ep;
      ep.pend = pend; ep.pth = w.pth;
      if constexpr (kKeepTwiddles) {
        NoPrefetchWrap<LoadPruned<kThreads, L, LOGI, RM>> lpw{lp};
        fft_run<kThreads, L, LOGI, +1, RM>(buf, rtid, lpw, ep, twb);
      } else {
        fft_run<kThreads, L, LOGI, +1, RM>(buf, rtid, lp, ep, twb);
      }
      __syncthreads();
      tx_epilogue<IO, kThreads, L, LOGI, RM>(ep, pend, w, at<IO>(a.out, B.t0), T.accumulate != 0, rtid);
      prev_end = T.ola ? B.t0 + N : INT64_MIN;
    }
  }
}

// Several subbands share the long IFFT: their weighted bands are added into
// one N-bin spectrum, then a full N-point IFFT. Short FFTs are dispatched by
// size in separate loops (one region per size keeps register use low).
template <int IO, int NL, bool FRONT>
__global__ __launch_bounds__(kThreads) void fc_tx_full_kernel(LaunchArgs a, int lmax) {
  extern __shared__ float2 smem[];
  const int task = blockIdx.x;
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  if (!T.accumulate) {
    zero_span<IO>(a.out, T.z0_lo, T.z0_hi);
    zero_span<IO>(a.out, T.z1_lo, T.z1_hi);
  }
  float2* S = smem;                                  // N-bin spectrum, then the in-place IFFT
  float2* bs = smem + lds_elems(NL);                 // short FFT scratch
  float2* pend = bs + lds_elems(lmax);               // OLA carry (N/2)
  const float2* tw = reinterpret_cast<const float2*>(a.twpass);
  const int tid = threadIdx.x;
  int64_t prev_end = INT64_MIN;
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    const int64_t next_start =
        (T.ola && bi + 1 < T.blk_count) ? a.blk[T.blk_first + bi + 1].t0 : INT64_MAX;
    const TxWin w = tx_window(B, T, prev_end, next_start, NL);
    __syncthreads();
    for (int i = tid; i < NL; i += kThreads) S[i] = make_float2(0.f, 0.f);
    auto run_size = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL) continue;
          const BlockSb Z = a.bsb[B.bs + m];
          StoreAddLong<NL> st;
          st.S = S; st.D = a.weights + Sb.w_off; st.ph = make_float2(Z.ph.x, Z.ph.y); st.L = LL; st.q0 = Sb.q0;
          __syncthreads();
          if constexpr (FRONT) {
            LoadGridRow<IO, LL> lg;
            lg.row = at<IO>(a.in, Z.x0); lg.K = Z.K;
            StoreScaled sx;
            sx.buf = bs; sx.scale = rsqrtf((float)LL);
            fft_run<kThreads, LL, 0, +1, radix_cap(LL)>(bs, tid, lg, sx, tw);
            __syncthreads();
            LoadCyclic<LL> lcy;
            lcy.x = bs; lcy.lo = Z.lo; lcy.hi = Z.hi; lcy.shift = Z.shift;
            fft_run<kThreads, LL, 0, -1, radix_cap(LL)>(bs, tid, lcy, st, tw);
          } else {
            LoadSeg<IO> ld;
            ld.x = at<IO>(a.in, Z.x0); ld.lo = Z.lo; ld.hi = Z.hi;
            fft_run<kThreads, LL, 0, -1, radix_cap(LL)>(bs, tid, ld, st, tw);
          }
        }
      }
    };
    run_size(SizeC<4096>()); run_size(SizeC<2048>()); run_size(SizeC<1024>()); run_size(SizeC<512>());
    run_size(SizeC<256>()); run_size(SizeC<128>()); run_size(SizeC<64>()); run_size(SizeC<32>());
    run_size(SizeC<16>()); run_size(SizeC<3072>()); run_size(SizeC<1536>()); run_size(SizeC<768>());
    __syncthreads();
    LoadLds ls;
    ls.s = S;
    TxEpiWin ep;
    ep.pend = pend; ep.pth = w.pth;
    ep.set_window(B.win, G.taper);
    fft_run<kThreads, NL, 0, +1, radix_cap(NL)>(S, tid, ls, ep, tw);
    __syncthreads();
    tx_epilogue<IO, kThreads, NL, 0, radix_cap(NL)>(ep, pend, w, at<IO>(a.out, B.t0), T.accumulate != 0,
                                                     (int)threadIdx.x);
    prev_end = T.ola ? B.t0 + NL : INT64_MIN;
  }
}

// ------------------------------------------------------------- RX tasks ---
// A run of consecutive blocks per task. Per block: the long FFT on the whole
// workgroup, whose last pass scatters every bin into the LDS region of each
// subband that gathers it (inverse-shift order; the regions overlay the
// spectrum); then each subband's short IFFT runs in place in its region:
// subbands with L <= 1024 as one-wave transforms on the wave the planner
// chose, longer ones on the whole workgroup. The next block's input is
// loaded into registers while the subbands run. Registers are bounded for
// four waves per SIMD (what the LDS allows at N = 4096); FP32 storage holds
// twice the prefetched input and would spill there (40 registers, 10 %
// slower than three waves without spills), so it takes three.
template <int IO, int NL, int TP>
__global__ __launch_bounds__(kThreads, IO == IO_C64 ? 3 : 4) void fc_rx_kernel(LaunchArgs a, int) {
  constexpr int RML = rx_long_cap(NL, TP);                 // long-FFT radix plan (transform plan TP)
  extern __shared__ float2 smem[];
  // consecutive tasks (runs sharing input at their boundary) go to the same
  // XCD: the dispatcher places workgroup i on XCD i mod 8
  const int n = gridDim.x;
  int task = blockIdx.x;
  if ((n & 7) == 0) task = (blockIdx.x & 7) * (n >> 3) + (blockIdx.x >> 3);
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  float2* S = smem;                                        // long spectrum, then subband regions
  const int tid = threadIdx.x, lane = tid & 63;
  // the planner's per-wave subband loads differ; rotating them with the
  // workgroup index keeps the heaviest from landing on the same SIMD in every
  // workgroup (the waves of a workgroup are spread over the CU's SIMDs in order)
  const int wave = ((tid >> 6) + blockIdx.x) & 3;
  const float2* tw = reinterpret_cast<const float2*>(a.twpass);
  const uint64_t* map = a.rxmap + G.map_off;
  LoadAhead<IO, kThreads, NL, RML> lh;
  {
    const BlockDesc B0 = a.blk[T.blk_first];
    lh.issue(at<IO>(a.in, B0.t0), B0.hlo, B0.hhi, tid);
  }
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    StoreScatter sc;
    sc.S = S; sc.map = map;
    __syncthreads();
    fft_run<kThreads, NL, 0, -1, RML>(S, tid, lh, sc, tw);
    if (bi + 1 < T.blk_count) {
      const BlockDesc Bn = a.blk[T.blk_first + bi + 1];
      lh.issue(at<IO>(a.in, Bn.t0), Bn.hlo, Bn.hhi, tid);
    }
    __syncthreads();
    auto run_wave = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave != wave) continue;
          const BlockSb Z = a.bsb[B.bs + m];
          StoreLow<IO> so;
          so.out = at<IO>(a.out, Z.x0); so.lo = Z.lo; so.hi = Z.hi; so.acc = T.accumulate != 0;
          so.ph = make_float2(Z.ph.x, Z.ph.y);
          LoadCompact<64, LL> lc2;
          lc2.R = S + Sb.cofs; lc2.D = a.weights + Sb.w_off;
          fft_run<64, LL, 0, +1, wave_radix_cap(LL)>(S + Sb.cofs, lane, lc2, so, tw);
        }
      }
    };
    run_wave(SizeC<1024>()); run_wave(SizeC<512>()); run_wave(SizeC<256>()); run_wave(SizeC<128>());
    run_wave(SizeC<64>()); run_wave(SizeC<32>()); run_wave(SizeC<16>()); run_wave(SizeC<768>());
    auto run_group = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave >= 0) continue;
          const BlockSb Z = a.bsb[B.bs + m];
          StoreLow<IO> so;
          so.out = at<IO>(a.out, Z.x0); so.lo = Z.lo; so.hi = Z.hi; so.acc = T.accumulate != 0;
          so.ph = make_float2(Z.ph.x, Z.ph.y);
          LoadCompact<kThreads, LL> lc2;
          lc2.R = S + Sb.cofs; lc2.D = a.weights + Sb.w_off;
          __syncthreads();
          fft_run<kThreads, LL, 0, +1, radix_cap(LL)>(S + Sb.cofs, tid, lc2, so, tw);
        }
      }
    };
    if (G.n_long_sb > 0) {
      run_group(SizeC<2048>());
      run_group(SizeC<4096>());
      run_group(SizeC<1536>());
      run_group(SizeC<3072>());
    }
  }
}

// ------------------------------------------------ demodulating RX -------
// v * j^k for k = 0..3.
__device__ __forceinline__ float2 rot_j(float2 v, int k) {
  const float2 r = (k & 1) ? make_float2(-v.y, v.x) : v;
  return (k & 2) ? make_float2(-r.x, -r.y) : r;
}

// First pass of the per-symbol IFFT, in place in the subband's region:
// V[u] = A[u] - B[u] with A[u] = g0[u] j^u from the first block's spectrum
// in the region and B[u] = g1[u] (-j)^u stored after the second block (GB:
// in device scratch at u, fetched with the weights before the pass; else in
// LDS at the padded position).
template <int NT, int L, int RM, bool GB> struct LoadV {
  const float2* R; const float2* B; const float* D; float2 ph;
  float d[16]; float2 b[GB ? 16 : 1];
  __device__ __forceinline__ void prefetch(int tid) {
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      int u, bb;
      if (first_pos<NT, L, 0, RM>(s, tid, u, bb)) {
        d[s] = D[wrap(u + (L >> 1), L)];
        if constexpr (GB) b[s] = B[u];
      }
    }
  }
  __device__ __forceinline__ float2 operator()(int slot, int u, int, int up) const {
    const float2 g0 = cscale(cmul(R[up], ph), d[slot]);
    return csub(rot_j(g0, u & 3), GB ? b[GB ? slot : 0] : B[up]);
  }
};

// Last pass of that IFFT: the half-band window keeps the first L/2 samples
// (and applies the inverse transform's 1/L).
struct StoreMask : NoPrefetch {
  float2* A; int half; float inv_l;
  __device__ __forceinline__ void operator()(int, int t, float2 v, int tp) const {
    A[tp] = t < half ? make_float2(v.x * inv_l, v.y * inv_l) : make_float2(0.f, 0.f);
  }
};

// First pass of the FFT back: the windowed samples in place.
struct LoadPadded : NoPrefetch {
  const float2* A;
  __device__ __forceinline__ float2 operator()(int, int, int, int ip) const { return A[ip]; }
};

// Last pass of that FFT: x[u] = (C V)[u] + B[u], scaled by 1/sqrt(L), to the
// symbol's subcarrier u (B from the scratch slot or the second region set).
template <int IO, int NT, int L, int RM, bool GB> struct StoreSubcarriers : NoPrefetch {
  const float2* B; typename Io<IO>::T* out; float scale;
  __device__ __forceinline__ void operator()(int, int u, float2 v, int up) const {
    const float2 x = cadd(v, B[GB ? u : up]);
    Io<IO>::st(out, u, make_float2(x.x * scale, x.y * scale));
  }
};

// The FFT back with its last pass's B loads and subcarrier stores through
// restrict-qualified pointers: within the call the compiler knows that the
// scratch B and the output do not overlap, so it issues the B loads ahead
// of the earlier stores instead of each after the store before it (with B in
// device scratch: 1.58 -> 1.51 ms on the 100 MHz bank, registers unchanged).
template <int IO, int NT, int LL, int RM, bool GB>
__device__ __forceinline__ void rxd_back(float2* R, int t, const float2* __restrict__ B,
                                         typename Io<IO>::T* __restrict__ out, float scale,
                                         const float2* tw) {
  LoadPadded lp;
  lp.A = R;
  StoreSubcarriers<IO, NT, LL, RM, GB> so;
  so.B = B; so.out = out; so.scale = scale;
  fft_run<NT, LL, 0, -1, RM>(R, t, lp, so, tw);
}

// Synchronised RX with OFDM demodulation in the simplified joint form of
// Sec. V-A. Tasks hold whole symbols (block pairs). Per symbol: the second
// block's long FFT is scattered into the subband regions and every subband
// stores B[u] = g1[u] (-j)^u, in a second region set above the spectrum, or
// (GB) in the task's scratch slot in device memory where the two sets would
// cost workgroups per CU (the filter bank's regions take 38.5 KB: two sets
// let two workgroups share a CU, one set three); the first block's long FFT
// is scattered likewise, then each subband runs V = A - B -> IFFT -> keep the
// first half -> FFT -> + B in place in its region and writes the L
// subcarriers. Subbands with L <= 1024 run on one wave (assignment as the RX
// kernel, the same wave storing and reading a subband's B), longer ones on
// the workgroup.
template <int IO, int NL, int TP, bool GB>
__global__ __launch_bounds__(kThreads, rxd_waves_per_simd(IO)) void fc_rxd_kernel(LaunchArgs a, int) {
  constexpr int RML = rx_long_cap(NL, TP);                 // long-FFT radix plan (transform plan TP)
  extern __shared__ float2 smem[];
  const int n = gridDim.x;
  int task = blockIdx.x;
  if ((n & 7) == 0) task = (blockIdx.x & 7) * (n >> 3) + (blockIdx.x >> 3);
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  float2* S = smem;                                        // spectrum, then the block's regions
  // B terms: the task's scratch slot (at aofs + u) or the second region set
  // (at scr_off + cofs + pad(u))
  float2* Bt = GB ? reinterpret_cast<float2*>(a.part + T.part_off) : smem + G.scr_off;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = ((tid >> 6) + blockIdx.x) & 3;
  const float2* tw = reinterpret_cast<const float2*>(a.twpass);
  const uint64_t* map = a.rxmap + G.map_off;
  LoadAhead<IO, kThreads, NL, RML> lh;
  {
    const BlockDesc B1 = a.blk[T.blk_first + 1];
    lh.issue(at<IO>(a.in, B1.t0), B1.hlo, B1.hhi, tid);
  }
  for (int bi = 0; bi + 1 < T.blk_count; bi += 2) {
    const BlockDesc B0 = a.blk[T.blk_first + bi];
    const BlockDesc B1 = a.blk[T.blk_first + bi + 1];
    StoreScatter sc;
    sc.S = S; sc.map = map;
    // ---- second block: spectrum -> regions -> B to the scratch slot
    __syncthreads();
    fft_run<kThreads, NL, 0, -1, RML>(S, tid, lh, sc, tw);
    lh.issue(at<IO>(a.in, B0.t0), B0.hlo, B0.hhi, tid);
    __syncthreads();
    for (int m = 0; m < G.n_sb; ++m) {
      const SbDesc Sb = a.sb[G.sb_first + m];
      const bool mine = Sb.wave >= 0 ? Sb.wave == wave : true;
      if (!mine) continue;
      const int step = Sb.wave >= 0 ? 64 : kThreads;
      const float2 ph = make_float2(a.bsb[B1.bs + m].ph.x, a.bsb[B1.bs + m].ph.y);
      const float* D = a.weights + Sb.w_off;
      const float2* R = S + Sb.cofs;
      float2* Bm = Bt + (GB ? Sb.aofs : Sb.cofs);
      for (int u = Sb.wave >= 0 ? lane : tid; u < Sb.L; u += step)
        Bm[GB ? u : pad(u)] = rot_j(cscale(cmul(R[pad(u)], ph), D[wrap(u + (Sb.L >> 1), Sb.L)]), (-u) & 3);
    }
    // (the barrier also orders the workgroup-wide subbands' B stores before
    // their reads by other threads)
    __syncthreads();
    // ---- first block: spectrum -> regions; per subband the joint transform
    fft_run<kThreads, NL, 0, -1, RML>(S, tid, lh, sc, tw);
    if (bi + 2 < T.blk_count) {
      const BlockDesc Bn = a.blk[T.blk_first + bi + 3];
      lh.issue(at<IO>(a.in, Bn.t0), Bn.hlo, Bn.hhi, tid);
    }
    __syncthreads();
    auto run_wave = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave != wave) continue;
          float2* R = S + Sb.cofs;
          const float2* Bm = Bt + (GB ? Sb.aofs : Sb.cofs);
          constexpr int RMW = wave_radix_cap(LL);
          LoadV<64, LL, RMW, GB> lv;
          lv.R = R; lv.B = Bm; lv.D = a.weights + Sb.w_off;
          lv.ph = make_float2(a.bsb[B0.bs + m].ph.x, a.bsb[B0.bs + m].ph.y);
          StoreMask sm;
          sm.A = R; sm.half = LL / 2; sm.inv_l = 1.f / LL;
          fft_run<64, LL, 0, +1, RMW>(R, lane, lv, sm, tw);
          wave_sync();
          rxd_back<IO, 64, LL, RMW, GB>(R, lane, Bm, at<IO>(a.out, a.bsb[B1.bs + m].x0), rsqrtf((float)LL), tw);
        }
      }
    };
    run_wave(SizeC<1024>()); run_wave(SizeC<512>()); run_wave(SizeC<256>()); run_wave(SizeC<128>());
    run_wave(SizeC<64>()); run_wave(SizeC<32>()); run_wave(SizeC<16>()); run_wave(SizeC<768>());
    auto run_group = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave >= 0) continue;
          float2* R = S + Sb.cofs;
          const float2* Bm = Bt + (GB ? Sb.aofs : Sb.cofs);
          constexpr int RMG = radix_cap(LL);
          LoadV<kThreads, LL, RMG, GB> lv;
          lv.R = R; lv.B = Bm; lv.D = a.weights + Sb.w_off;
          lv.ph = make_float2(a.bsb[B0.bs + m].ph.x, a.bsb[B0.bs + m].ph.y);
          StoreMask sm;
          sm.A = R; sm.half = LL / 2; sm.inv_l = 1.f / LL;
          __syncthreads();
          fft_run<kThreads, LL, 0, +1, RMG>(R, tid, lv, sm, tw);
          __syncthreads();
          rxd_back<IO, kThreads, LL, RMG, GB>(R, tid, Bm, at<IO>(a.out, a.bsb[B1.bs + m].x0), rsqrtf((float)LL),
                                             tw);
        }
      }
    };
    if (G.n_long_sb > 0) {
      run_group(SizeC<2048>());
      run_group(SizeC<4096>());
      run_group(SizeC<1536>());
      run_group(SizeC<3072>());
    }
  }
}

// ---------------------------------------------------- weight gradient ---
// Last pass of the short FFT of the forward input block: bin u (natural
// order, weight index p = (u + L/2) mod L) adds Re(conj(A) X) to its LDS
// accumulator, where A = G(Xi(p)) * phase is the adjoint's value for that bin
// before the weight (G the long FFT of the gradient block, held in the
// subband's region) and X the forward short-FFT bin.
struct StoreGrad : NoPrefetch {
  const float2* R; float2 ph; float* acc;
  __device__ __forceinline__ void operator()(int, int u, float2 x, int up) const {
    const float2 a = cmul(R[up], ph);
    acc[u] += a.x * x.x + a.y * x.y;
  }
};

// The same with each thread's sums in registers: output slot s of the last
// pass is bin last_pos(s) in every block, so the thread that produces a bin
// is the one that accumulates it.
struct StoreGradReg : NoPrefetch {
  const float2* R; float2 ph; float r[16];
  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int s = 0; s < 16; ++s) r[s] = 0.f;
  }
  __device__ __forceinline__ void operator()(int slot, int, float2 x, int up) {
    const float2 a = cmul(R[up], ph);
    r[slot] += a.x * x.x + a.y * x.y;
  }
};

// Per block, as the adjoint: long FFT of the gradient block scattered into
// the subband regions; then per subband the short FFT of the forward input
// block (window and phase of the forward transform) in a scratch buffer,
// whose last pass accumulates the products. Each sum belongs to one thread
// for the whole task (in registers for one-subband groups, in LDS for groups
// of several subbands); at the end the task stores its sums in its own
// partial-sum slot (TaskDesc::part_off), in weight order, and
// fc_wgrad_reduce_kernel adds the slots of each group in block order: no
// atomics, so grad_w does not depend on the work split or launch order.
template <int IO, int NL>
__global__ __launch_bounds__(kThreads) void fc_wgrad_kernel(LaunchArgs a, int) {
  extern __shared__ float2 smem[];
  const int n = gridDim.x;
  int task = blockIdx.x;
  if ((n & 7) == 0) task = (blockIdx.x & 7) * (n >> 3) + (blockIdx.x >> 3);
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  float2* S = smem;
  float2* scr = smem + G.scr_off;
  float* acc = reinterpret_cast<float*>(smem + G.acc_off);
  const int tid = threadIdx.x, lane = tid & 63;
  // the planner's per-wave subband loads differ; rotating them with the
  // workgroup index keeps the heaviest from landing on the same SIMD in every
  // workgroup (the waves of a workgroup are spread over the CU's SIMDs in order)
  const int wave = ((tid >> 6) + blockIdx.x) & 3;
  const float2* tw = reinterpret_cast<const float2*>(a.twpass);
  const uint64_t* map = a.rxmap + G.map_off;
  LoadAhead<IO, kThreads, NL, radix_cap(NL)> lh;
  {
    const BlockDesc B0 = a.blk[T.blk_first];
    lh.issue(at<IO>(a.in, B0.t0), B0.hlo, B0.hhi, tid);
  }
  if (G.wg_nb > 0) {
    // one subband, L <= 1024: the long FFTs of a group of blocks scatter into
    // one band region each, then every wave runs the short FFT of one
    // block's forward input against its region. Each lane keeps the sums of
    // its own bins in registers (the same bins in every block); at the end
    // the waves' sums meet in LDS.
    const SbDesc Sb = a.sb[G.sb_first];
    const int L = Sb.L, NBG = G.wg_nb, le = lds_elems(L);
    float2* reg = S + lds_elems(NL);
    float2* sbuf = reg + NBG * le;
    StoreGradReg sg;
    sg.clear();
    // this wave's forward-input block of the group, loaded while the group's
    // long FFTs run
    LoadAhead<IO, 64, 1024> lx;
    for (int g0 = 0; g0 < T.blk_count; g0 += NBG) {
      const int nb = T.blk_count - g0 < NBG ? T.blk_count - g0 : NBG;
      if (wave < nb) {
        const BlockSb Z = a.bsb[a.blk[T.blk_first + g0 + wave].bs];
        auto issue = [&](auto lc) {
          constexpr int LL = decltype(lc)::value;
          if constexpr (divides_pow2(LL, NL)) {
            if (L == LL) lx.template issue_sized<LL, wave_radix_cap(LL)>(at<IO>(a.in2, Z.x0), Z.lo, Z.hi, lane);
          }
        };
        issue(SizeC<1024>()); issue(SizeC<512>()); issue(SizeC<256>()); issue(SizeC<128>());
        issue(SizeC<64>()); issue(SizeC<32>()); issue(SizeC<16>()); issue(SizeC<768>());
      }
      for (int k = 0; k < nb; ++k) {
        StoreScatter sc;
        sc.S = reg + k * le; sc.map = map;
        __syncthreads();
        fft_run<kThreads, NL, 0, -1, radix_cap(NL)>(S, tid, lh, sc, tw);
        if (g0 + k + 1 < T.blk_count) {
          const BlockDesc Bn = a.blk[T.blk_first + g0 + k + 1];
          lh.issue(at<IO>(a.in, Bn.t0), Bn.hlo, Bn.hhi, tid);
        }
      }
      __syncthreads();
      if (wave < nb) {
        const BlockSb Z = a.bsb[a.blk[T.blk_first + g0 + wave].bs];
        auto run = [&](auto lc) {
          constexpr int LL = decltype(lc)::value;
          if constexpr (divides_pow2(LL, NL)) {
            if (L != LL) return;
            sg.R = reg + wave * le; sg.ph = make_float2(Z.ph.x, Z.ph.y);
            fft_run<64, LL, 0, -1, wave_radix_cap(LL)>(sbuf + wave * le, lane, lx, sg, tw);
          }
        };
        run(SizeC<1024>()); run(SizeC<512>()); run(SizeC<256>()); run(SizeC<128>());
        run(SizeC<64>()); run(SizeC<32>()); run(SizeC<16>()); run(SizeC<768>());
      }
    }
    __syncthreads();
    // the long-FFT buffer and the band regions after it are free now and
    // hold the NBG waves' sums (NBG L floats = NBG L / 2 complex entries)
    float* red = reinterpret_cast<float*>(S);
    if (wave < NBG) {
      auto put = [&](auto lc) {
        constexpr int LL = decltype(lc)::value;
        if constexpr (divides_pow2(LL, NL)) {
          if (L != LL) return;
#pragma unroll
          for (int s = 0; s < 16; ++s) {
            const int u = last_pos<64, LL, 0, wave_radix_cap(LL)>(s, lane);
            if (u >= 0) red[wave * LL + u] = sg.r[s];
          }
        }
      };
      put(SizeC<1024>()); put(SizeC<512>()); put(SizeC<256>()); put(SizeC<128>());
      put(SizeC<64>()); put(SizeC<32>()); put(SizeC<16>()); put(SizeC<768>());
    }
    __syncthreads();
    float* part = a.part + T.part_off + Sb.aofs;
    for (int u = tid; u < L; u += kThreads) {
      float sum = 0.f;
      for (int w = 0; w < NBG; ++w) sum += red[w * L + u];
      part[wrap(u + (L >> 1), L)] = sum;
    }
    return;
  }
  if (G.n_sb == 1 && G.n_long_sb == 1) {
    // one subband with a whole-workgroup short FFT (L > 1024): its forward
    // input block is loaded while the block's long FFT runs, and every thread
    // keeps the sums of its own bins in registers (these groups have launches
    // of their own, without the LDS accumulators)
    const SbDesc Sb = a.sb[G.sb_first];
    auto run = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL) && LL > 1024) {
        if (Sb.L != LL) return;
        constexpr int RML = radix_cap(LL);
        StoreGradReg sg;
        sg.clear();
        LoadAhead<IO, kThreads, LL, RML> lx;
        for (int bi = 0; bi < T.blk_count; ++bi) {
          const BlockDesc B = a.blk[T.blk_first + bi];
          const BlockSb Z = a.bsb[B.bs];
          lx.issue(at<IO>(a.in2, Z.x0), Z.lo, Z.hi, tid);
          StoreScatter sc;
          sc.S = S; sc.map = map;
          __syncthreads();
          fft_run<kThreads, NL, 0, -1, radix_cap(NL)>(S, tid, lh, sc, tw);
          if (bi + 1 < T.blk_count) {
            const BlockDesc Bn = a.blk[T.blk_first + bi + 1];
            lh.issue(at<IO>(a.in, Bn.t0), Bn.hlo, Bn.hhi, tid);
          }
          __syncthreads();
          sg.R = S + Sb.cofs; sg.ph = make_float2(Z.ph.x, Z.ph.y);
          fft_run<kThreads, LL, 0, -1, RML>(scr, tid, lx, sg, tw);
        }
        float* part = a.part + T.part_off + Sb.aofs;
#pragma unroll
        for (int s = 0; s < 16; ++s) {
          const int u = last_pos<kThreads, LL, 0, RML>(s, tid);
          if (u >= 0) part[wrap(u + (LL >> 1), LL)] = sg.r[s];
        }
      }
    };
    run(SizeC<2048>()); run(SizeC<4096>()); run(SizeC<1536>()); run(SizeC<3072>());
    return;
  }
  for (int i = tid; i < G.acc_len; i += kThreads) acc[i] = 0.f;
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    StoreScatter sc;
    sc.S = S; sc.map = map;
    __syncthreads();
    fft_run<kThreads, NL, 0, -1, radix_cap(NL)>(S, tid, lh, sc, tw);
    if (bi + 1 < T.blk_count) {
      const BlockDesc Bn = a.blk[T.blk_first + bi + 1];
      lh.issue(at<IO>(a.in, Bn.t0), Bn.hlo, Bn.hhi, tid);
    }
    __syncthreads();
    auto run_wave = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave != wave) continue;
          const BlockSb Z = a.bsb[B.bs + m];
          LoadSeg<IO> ls;
          ls.x = at<IO>(a.in2, Z.x0); ls.lo = Z.lo; ls.hi = Z.hi;
          StoreGrad sg;
          sg.R = S + Sb.cofs; sg.ph = make_float2(Z.ph.x, Z.ph.y); sg.acc = acc + Sb.aofs;
          wave_sync();
          fft_run<64, LL, 0, -1, wave_radix_cap(LL)>(scr + wave * G.wstride, lane, ls, sg, tw);
        }
      }
    };
    run_wave(SizeC<1024>()); run_wave(SizeC<512>()); run_wave(SizeC<256>()); run_wave(SizeC<128>());
    run_wave(SizeC<64>()); run_wave(SizeC<32>()); run_wave(SizeC<16>()); run_wave(SizeC<768>());
    auto run_group = [&](auto lc) {
      constexpr int LL = decltype(lc)::value;
      if constexpr (divides_pow2(LL, NL)) {
        for (int m = 0; m < G.n_sb; ++m) {
          const SbDesc Sb = a.sb[G.sb_first + m];
          if (Sb.L != LL || Sb.wave >= 0) continue;
          const BlockSb Z = a.bsb[B.bs + m];
          StoreGrad sg;
          sg.R = S + Sb.cofs; sg.ph = make_float2(Z.ph.x, Z.ph.y); sg.acc = acc + Sb.aofs;
          __syncthreads();
          LoadSeg<IO> ls;
          ls.x = at<IO>(a.in2, Z.x0); ls.lo = Z.lo; ls.hi = Z.hi;
          fft_run<kThreads, LL, 0, -1, radix_cap(LL)>(scr, tid, ls, sg, tw);
        }
      }
    };
    if (G.n_long_sb > 0) {
      run_group(SizeC<2048>());
      run_group(SizeC<4096>());
      run_group(SizeC<1536>());
      run_group(SizeC<3072>());
    }
  }
  __syncthreads();
  float* part = a.part + T.part_off;
  for (int m = 0; m < G.n_sb; ++m) {
    const SbDesc Sb = a.sb[G.sb_first + m];
    for (int u = tid; u < Sb.L; u += kThreads) part[Sb.aofs + wrap(u + (Sb.L >> 1), Sb.L)] = acc[Sb.aofs + u];
  }
}

// grad_w of every subband of group blockIdx.x: the sum of the group's task
// slots, taken in block order (a fixed order, so the result is the same for
// every work split and launch order). Every weight is written. (The sums do
// not depend on the I/O type; one instance per type keeps the dispatch
// uniform.)
template <int IO>
__global__ __launch_bounds__(kThreads) void fc_wgrad_reduce_kernel(const SbDesc* sb, const GroupDesc* grp,
                                                                     int n_grp, const float* part, float* gw) {
  const int g = blockIdx.x;
  if (g >= n_grp) return;
  const GroupDesc G = grp[g];
  for (int m = 0; m < G.n_sb; ++m) {
    const SbDesc Sb = sb[G.sb_first + m];
    const float* p0 = part + G.part_base + Sb.aofs;
    for (int p = threadIdx.x; p < Sb.L; p += kThreads) {
      float sum = 0.f;
      for (int t = 0; t < G.part_n; ++t) sum += p0[(int64_t)t * G.acc_len + p];
      gw[Sb.w_off + p] = sum;
    }
  }
}

template <int IO>
__global__ __launch_bounds__(kThreads) void fc_zero_kernel(void* out, int64_t n) {
  typename Io<IO>::T* p = at<IO>(out, 0);
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    Io<IO>::st(p + i, 0, make_float2(0.f, 0.f));
}

// ------------------------------------------------------ per-I/O dispatch ---
// Kernel classes: 0 = TX pruned (size = L, aux = log2 I), 1 = TX full
// (size = N, aux = largest L), 2 = RX and adjoint (size = N), 3 = weight
// gradient (size = N), 4 = demodulating RX (size = N), 5 = weight-gradient
// reduction (one workgroup per group, n_task = number of groups).
// One pruned-TX instance: transform plan a.tplan where the size has a second
// plan (pruned_has_alt), else plan 0.
template <int IO, int L, int LI>
hipError_t launch_pruned_li(const LaunchArgs& a, size_t lds, hipStream_t s, dim3 grid) {
  dim3 block(kThreads);
  if constexpr (pruned_has_alt(L)) {
    if (a.tplan) {
      if (a.front) hipLaunchKernelGGL((fc_tx_pruned_kernel<IO, L, LI, true, 1>), grid, block, lds, s, a);
      else hipLaunchKernelGGL((fc_tx_pruned_kernel<IO, L, LI, false, 1>), grid, block, lds, s, a);
      return hipGetLastError();
    }
  }
  if (a.front) hipLaunchKernelGGL((fc_tx_pruned_kernel<IO, L, LI, true, 0>), grid, block, lds, s, a);
  else hipLaunchKernelGGL((fc_tx_pruned_kernel<IO, L, LI, false, 0>), grid, block, lds, s, a);
  return hipGetLastError();
}

template <int IO, int L>
hipError_t launch_pruned(const LaunchArgs& a, int logi, size_t lds, hipStream_t s, dim3 grid) {
  switch (logi) {
#define FC_LI(LI) \
  case LI:                                                                                          \
    if constexpr ((L << LI) <= kMaxPoints) return launch_pruned_li<IO, L, LI>(a, lds, s, grid);      \
    break;
    FC_LI(1) FC_LI(2) FC_LI(3) FC_LI(4) FC_LI(5) FC_LI(6) FC_LI(7) FC_LI(8)
#undef FC_LI
    default: break;
  }
  return hipErrorInvalidValue;
}

template <int IO, int SZ>
hipError_t launch_size(int cls, const LaunchArgs& a, int aux, size_t lds, hipStream_t s, dim3 grid) {
  dim3 block(kThreads);
  if (cls == 0) {
    if constexpr (is_pow2c(SZ)) return launch_pruned<IO, SZ>(a, aux, lds, s, grid);
    else return hipErrorInvalidValue;        // mixed-radix groups use the full-transform kernel
  }
  // the RX family under transform plan a.tplan where the size has a second plan
  constexpr bool alt = rx_has_alt(SZ);
  if (cls == 1) {
    if (a.front) hipLaunchKernelGGL((fc_tx_full_kernel<IO, SZ, true>), grid, block, lds, s, a, aux);
    else hipLaunchKernelGGL((fc_tx_full_kernel<IO, SZ, false>), grid, block, lds, s, a, aux);
  } else if (cls == 3) {
    hipLaunchKernelGGL((fc_wgrad_kernel<IO, SZ>), grid, block, lds, s, a, aux);
  } else if (cls == 4) {
    // aux: 1 = the B terms in device scratch
    if (aux) {
      if (alt && a.tplan) hipLaunchKernelGGL((fc_rxd_kernel<IO, SZ, alt ? 1 : 0, true>), grid, block, lds, s, a, aux);
      else hipLaunchKernelGGL((fc_rxd_kernel<IO, SZ, 0, true>), grid, block, lds, s, a, aux);
    } else {
      if (alt && a.tplan) hipLaunchKernelGGL((fc_rxd_kernel<IO, SZ, alt ? 1 : 0, false>), grid, block, lds, s, a, aux);
      else hipLaunchKernelGGL((fc_rxd_kernel<IO, SZ, 0, false>), grid, block, lds, s, a, aux);
    }
  } else {
    if (alt && a.tplan) hipLaunchKernelGGL((fc_rx_kernel<IO, SZ, alt ? 1 : 0>), grid, block, lds, s, a, aux);
    else hipLaunchKernelGGL((fc_rx_kernel<IO, SZ, 0>), grid, block, lds, s, a, aux);
  }
  return hipGetLastError();
}

template <int IO>
hipError_t launch_io(int cls, int size, const LaunchArgs& a, int aux, size_t lds, hipStream_t s) {
  if (a.n_task <= 0) return hipSuccess;
  if (cls == 5) {
    hipLaunchKernelGGL(fc_wgrad_reduce_kernel<IO>, dim3(a.n_task), dim3(kThreads), 0, s, a.sb, a.grp, a.n_task,
                       a.part, reinterpret_cast<float*>(a.out));
    return hipGetLastError();
  }
  dim3 grid(cls >= 2 ? ((a.n_task + 7) & ~7) : a.n_task);
  switch (size) {
#define FC_SZ(SZ) case SZ: return launch_size<IO, SZ>(cls, a, aux, lds, s, grid);
    FC_SZ(16) FC_SZ(32) FC_SZ(64) FC_SZ(128) FC_SZ(256) FC_SZ(512) FC_SZ(1024) FC_SZ(2048) FC_SZ(4096)
    FC_SZ(768) FC_SZ(1536) FC_SZ(3072)
#undef FC_SZ
    default: return hipErrorInvalidValue;
  }
}

template <int IO>
hipError_t launch_zero_io(void* out, int64_t n, hipStream_t s) {
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fc_zero_kernel<IO>, dim3((unsigned)blocks), dim3(kThreads), 0, s, out, n);
  return hipGetLastError();
}

template <class K>
void grant_lds(K* kernel, size_t bytes, hipError_t& e) {
  const hipError_t r = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (r != hipSuccess) e = r;
}

template <int IO, int L>
void lds_limit_pruned(size_t bytes, hipError_t& e) {
#define FC_LI(LI)                                                                                   \
  if constexpr ((L << LI) <= kMaxPoints) {                                                          \
    grant_lds(fc_tx_pruned_kernel<IO, L, LI, false, 0>, bytes, e);                                  \
    grant_lds(fc_tx_pruned_kernel<IO, L, LI, true, 0>, bytes, e);                                   \
    if constexpr (pruned_has_alt(L)) {                                                              \
      grant_lds(fc_tx_pruned_kernel<IO, L, LI, false, 1>, bytes, e);                                \
      grant_lds(fc_tx_pruned_kernel<IO, L, LI, true, 1>, bytes, e);                                 \
    }                                                                                               \
  }
  FC_LI(1) FC_LI(2) FC_LI(3) FC_LI(4) FC_LI(5) FC_LI(6) FC_LI(7) FC_LI(8)
#undef FC_LI
}

template <int IO, int SZ>
void lds_limits_size(size_t bytes, hipError_t& e) {
  if constexpr (is_pow2c(SZ)) lds_limit_pruned<IO, SZ>(bytes, e);
  grant_lds(fc_tx_full_kernel<IO, SZ, false>, bytes, e);
  grant_lds(fc_tx_full_kernel<IO, SZ, true>, bytes, e);
  grant_lds(fc_rx_kernel<IO, SZ, 0>, bytes, e);
  grant_lds(fc_rxd_kernel<IO, SZ, 0, false>, bytes, e);
  grant_lds(fc_rxd_kernel<IO, SZ, 0, true>, bytes, e);
  if constexpr (rx_has_alt(SZ)) {
    grant_lds(fc_rx_kernel<IO, SZ, 1>, bytes, e);
    grant_lds(fc_rxd_kernel<IO, SZ, 1, false>, bytes, e);
    grant_lds(fc_rxd_kernel<IO, SZ, 1, true>, bytes, e);
  }
  grant_lds(fc_wgrad_kernel<IO, SZ>, bytes, e);
}

template <int IO>
hipError_t lds_limits_io(size_t bytes) {
  hipError_t e = hipSuccess;
  lds_limits_size<IO, 16>(bytes, e); lds_limits_size<IO, 32>(bytes, e); lds_limits_size<IO, 64>(bytes, e);
  lds_limits_size<IO, 128>(bytes, e); lds_limits_size<IO, 256>(bytes, e); lds_limits_size<IO, 512>(bytes, e);
  lds_limits_size<IO, 1024>(bytes, e); lds_limits_size<IO, 2048>(bytes, e); lds_limits_size<IO, 4096>(bytes, e);
  lds_limits_size<IO, 768>(bytes, e); lds_limits_size<IO, 1536>(bytes, e); lds_limits_size<IO, 3072>(bytes, e);
  return e;
}

}  // namespace fcx

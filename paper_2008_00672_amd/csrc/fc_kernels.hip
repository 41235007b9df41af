// gfx950 kernels of the fast-convolution (FC) filter banks.
//
// One workgroup (256 threads, 4 wave64) processes one task: a run of
// consecutive FC blocks of one processing group (TX) or one block (RX).
// Transforms are Stockham FFTs held in LDS: every pass loads R values per
// butterfly into registers, applies the inter-pass twiddles (FP32 table built
// in FP64 on the host), runs a radix-R (2/4/8/16) DFT in registers and writes
// back in place after a barrier. Up to 16 complex values per thread, so one
// workgroup holds transforms of up to 4096 points (or batches of shorter ones
// with the same total). The first pass reads through a load functor (global
// memory or another LDS array) and the last pass hands its results to a store
// functor in registers, so segmentation, windowing, bin mapping, weighting and
// the overlap-add / overlap-save combination are fused into the transforms.
//
// Paper: Yli-Kaakinen et al., arXiv 2008.00672. TX follows the block operator
// W_N^{-1} M(phi) D P^(L/2) W_L A (Sec. III-B) and its symbol-synchronised
// form (Sec. III-C..III-E); RX follows W_L^{-1} P^(-L/2) D M^T W_N (Sec. IV).
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

// ------------------------------------------------------------ pass plan ---
constexpr int log2i(int n) { return n <= 1 ? 0 : 1 + log2i(n >> 1); }
constexpr int npass(int P) { return P <= 16 ? 1 : (P <= 256 ? 2 : 3); }
constexpr int radix_of(int P, int s) {
  // 2..16: one pass; 32..256: two; 512..4096: three
  return P <= 16 ? P
       : P == 32 ? (s == 0 ? 8 : 4)
       : P == 64 ? 8
       : P == 128 ? (s == 0 ? 16 : 8)
       : P == 256 ? 16
       : P == 512 ? 8
       : P == 1024 ? (s < 2 ? 16 : 4)
       : P == 2048 ? (s < 2 ? 16 : 8)
       : 16;
}

// One Stockham pass over P-point transforms, Bt = 2^logBt of them interleaved
// (element i of transform b at index i * Bt + b).
template <int P, int R, int DIR, bool FIRST, bool LAST, class Load, class Store>
__device__ __forceinline__ void fft_pass(float2* __restrict__ buf, int logBt, int Ns, Load& load,
                                         Store& store, const float2* __restrict__ tw) {
  constexpr int NB = P / R;
  constexpr int MAXIT = 16 / R;
  const int total = NB << logBt;
  const int bmask = (1 << logBt) - 1;
  float2 v[MAXIT][R];
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int g = threadIdx.x + it * kThreads;
    if (g < total) {
      const int b = g & bmask, j = g >> logBt;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if constexpr (FIRST)
          v[it][r] = load(j + r * NB, b);
        else
          v[it][r] = buf[((j + r * NB) << logBt) + b];
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < MAXIT; ++it) {
    const int g = threadIdx.x + it * kThreads;
    if (g < total) {
      const int b = g & bmask, j = g >> logBt;
      const int k = j & (Ns - 1);
      if constexpr (!FIRST) {
        const int stride = kTwiddleN / (Ns * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[k * r * stride];
          if (DIR > 0) w.y = -w.y;
          v[it][r] = cmul(v[it][r], w);
        }
      }
      Dft<R, DIR>::run(v[it]);
      if constexpr (LAST) {
#pragma unroll
        for (int r = 0; r < R; ++r) store(it * R + r, ((j + r * NB) << logBt) + b, v[it][r]);
      } else {
        const int base = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[((base + r * Ns) << logBt) + b] = v[it][r];
      }
    }
  }
  if constexpr (!LAST) __syncthreads();
}

// Full transform: DIR = -1 forward DFT, +1 unnormalised inverse.
// Requires P * 2^logBt <= 4096 and a barrier before the call if `buf` (or what
// `load` reads) was written by other threads.
template <int P, int DIR, class Load, class Store>
__device__ __forceinline__ void fft_run(float2* buf, int logBt, Load& load, Store& store,
                                        const float2* __restrict__ tw) {
  constexpr int NP = npass(P);
  constexpr int R0 = radix_of(P, 0), R1 = radix_of(P, 1), R2 = radix_of(P, 2);
  fft_pass<P, R0, DIR, true, NP == 1>(buf, logBt, 1, load, store, tw);
  if constexpr (NP >= 2) fft_pass<P, R1, DIR, false, NP == 2>(buf, logBt, R0, load, store, tw);
  if constexpr (NP >= 3) fft_pass<P, R2, DIR, false, true>(buf, logBt, R0 * R1, load, store, tw);
}

// ------------------------------------------------------------------- I/O --
template <int IO> __device__ __forceinline__ float2 ld_io(const void* p, int64_t i);
template <> __device__ __forceinline__ float2 ld_io<IO_C64>(const void* p, int64_t i) {
  return reinterpret_cast<const float2*>(p)[i];
}
template <> __device__ __forceinline__ float2 ld_io<IO_F16>(const void* p, int64_t i) {
  return __half22float2(reinterpret_cast<const __half2*>(p)[i]);
}
template <> __device__ __forceinline__ float2 ld_io<IO_BF16>(const void* p, int64_t i) {
  const uint32_t u = reinterpret_cast<const uint32_t*>(p)[i];
  return make_float2(__uint_as_float(u << 16), __uint_as_float(u & 0xffff0000u));
}

__device__ __forceinline__ uint32_t f2bf_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;        // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <int IO> __device__ __forceinline__ void st_io(void* p, int64_t i, float2 v);
template <> __device__ __forceinline__ void st_io<IO_C64>(void* p, int64_t i, float2 v) {
  reinterpret_cast<float2*>(p)[i] = v;
}
template <> __device__ __forceinline__ void st_io<IO_F16>(void* p, int64_t i, float2 v) {
  reinterpret_cast<__half2*>(p)[i] = __float22half2_rn(v);
}
template <> __device__ __forceinline__ void st_io<IO_BF16>(void* p, int64_t i, float2 v) {
  reinterpret_cast<uint32_t*>(p)[i] = f2bf_rne(v.x) | (f2bf_rne(v.y) << 16);
}

template <int IO>
__device__ __forceinline__ void put(void* p, int64_t i, float2 v, bool acc) {
  if (acc) v = cadd(v, ld_io<IO>(p, i));
  st_io<IO>(p, i, v);
}

// ------------------------------------------------------------- functors ---
// Low-rate segment: sample i of the block is x[x0 + i] inside [lo, hi), else 0.
template <int IO> struct LoadSeg {
  const void* in; int64_t x0; int lo, hi;
  __device__ __forceinline__ float2 operator()(int i, int) const {
    return (i >= lo && i < hi) ? ld_io<IO>(in, x0 + i) : make_float2(0.f, 0.f);
  }
};

// Plain LDS read in interleaved order (used where the first pass reads LDS).
struct LoadLds {
  const float2* s; int logBt;
  __device__ __forceinline__ float2 operator()(int i, int b) const { return s[(i << logBt) + b]; }
};

// TX, pruned long IFFT: short-FFT bin u -> residue rho = (u + c) mod L of the
// band, weighted by D[p] (p = (u + L/2) mod L, the fftshifted index) and the
// block phase.
struct StoreBand {
  float2* V; const float* D; float2 ph; int L, c;
  __device__ __forceinline__ void operator()(int, int u, float2 v) const {
    const int p = (u + (L >> 1)) & (L - 1);
    V[(u + c) & (L - 1)] = cscale(cmul(v, ph), D[p]);
  }
};

// TX, pruned long IFFT first pass: sub-transform b (output samples t = a*Bt + b)
// of residue rho takes V[rho] * exp(+j 2 pi q b / N), q the band bin of rho.
struct LoadPruned {
  const float2* V; const float2* tw; int L, N, q0, twstep;
  __device__ __forceinline__ float2 operator()(int rho, int b) const {
    const int q = (q0 + ((rho - q0) & (L - 1))) & (N - 1);
    float2 w = tw[((q * b) & (N - 1)) * twstep];
    w.y = -w.y;
    return cmul(V[rho], w);
  }
};

// TX, full long IFFT: add the weighted band into the N-bin spectrum.
struct StoreAddLong {
  float2* S; const float* D; float2 ph; int L, N, q0;
  __device__ __forceinline__ void operator()(int, int u, float2 v) const {
    const int p = (u + (L >> 1)) & (L - 1);
    const int q = (q0 + p) & (N - 1);
    S[q] = cadd(S[q], cscale(cmul(v, ph), D[p]));
  }
};

// TX epilogue: OLA carry-in (phase 1, inside the last pass); results stay in
// registers until phase 2.
struct TxEpi {
  const float2* pend; int64_t t0, prev_end;
  float2 val[16];
  int pos[16];
  __device__ __forceinline__ void operator()(int slot, int t, float2 v) {
    if (t0 + t < prev_end) v = cadd(v, pend[t]);
    val[slot] = v;
    pos[slot] = t;
  }
};

// RX: long-FFT result into the LDS spectrum (natural order).
struct StoreLds {
  float2* s;
  __device__ __forceinline__ void operator()(int, int t, float2 v) const { s[t] = v; }
};

// High-rate segment with an input window [lo, hi).
template <int IO> struct LoadHigh {
  const void* in; int64_t t0; int lo, hi;
  __device__ __forceinline__ float2 operator()(int i, int) const {
    return (i >= lo && i < hi) ? ld_io<IO>(in, t0 + i) : make_float2(0.f, 0.f);
  }
};

// RX short IFFT first pass: bin u of the subband (inverse shift) gathers long
// bin q = (q0 + p) mod N, p = (u + L/2) mod L, weighted by D[p] and conj phase.
struct LoadGather {
  const float2* S; const float* D; float2 ph; int L, N, q0;
  __device__ __forceinline__ float2 operator()(int u, int) const {
    const int p = (u + (L >> 1)) & (L - 1);
    return cscale(cmul(S[(q0 + p) & (N - 1)], ph), D[p]);
  }
};

// RX output: keep window [lo, hi) of the low-rate block, at x0 + i.
template <int IO> struct StoreLow {
  void* out; int64_t x0; int lo, hi; bool acc;
  __device__ __forceinline__ void operator()(int, int i, float2 v) const {
    if (i >= lo && i < hi) put<IO>(out, x0 + i, v, acc);
  }
};

// ------------------------------------------------------------- TX tasks ---
template <int IO>
__device__ __forceinline__ void zero_range(void* out, int64_t lo, int64_t hi) {
  for (int64_t i = lo + threadIdx.x; i < hi; i += kThreads) st_io<IO>(out, i, make_float2(0.f, 0.f));
}

// Epilogue phase 2 (after a barrier): OLA carry-out or write the owned samples.
template <int IO>
__device__ __forceinline__ void tx_epilogue(TxEpi& ep, float2* pend, int64_t next_start, int hlo, int hhi,
                                            const TaskDesc& T, void* out) {
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int t = ep.pos[s];
    if (t < 0) continue;
    const int64_t ta = ep.t0 + t;
    if (ta >= next_start) {
      pend[ta - next_start] = ep.val[s];
    } else if (t >= hlo && t < hhi && ta >= T.own_lo && ta < T.own_hi) {
      put<IO>(out, ta, ep.val[s], T.accumulate != 0);
    }
  }
}

template <int IO, int L>
__device__ __forceinline__ void tx_task_pruned(const LaunchArgs& a, const TaskDesc& T, const GroupDesc& G, float2* smem) {
  const SbDesc S = a.sb[G.sb_first];
  const int N = G.N;
  const int logBt = G.logN - S.logL;
  float2* buf = smem;           // N points: short FFT, band V (first L) and the batched IFFT
  float2* pend = smem + N;      // OLA carry, up to N/2 points
  const float* D = a.weights + S.w_off;
  int64_t prev_end = INT64_MIN;
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    const BlockSb Z = a.bsb[B.bs];
    const int64_t next_start =
        (T.ola && bi + 1 < T.blk_count) ? a.blk[T.blk_first + bi + 1].t0 : INT64_MAX;
    LoadSeg<IO> ld{a.in, Z.x0, Z.lo, Z.hi};
    StoreBand sb{buf, D, make_float2(Z.ph.x, Z.ph.y), L, S.c};
    __syncthreads();
    fft_run<L, -1>(buf, 0, ld, sb, reinterpret_cast<const float2*>(a.twiddle));
    __syncthreads();
    LoadPruned lp{buf, reinterpret_cast<const float2*>(a.twiddle), L, N, S.q0, kTwiddleN / N};
    TxEpi ep;
    ep.pend = pend; ep.t0 = B.t0; ep.prev_end = prev_end;
#pragma unroll
    for (int s = 0; s < 16; ++s) ep.pos[s] = -1;
    fft_run<L, +1>(buf, logBt, lp, ep, reinterpret_cast<const float2*>(a.twiddle));
    __syncthreads();
    tx_epilogue<IO>(ep, pend, next_start, B.hlo, B.hhi, T, a.out);
    prev_end = T.ola ? B.t0 + N : INT64_MIN;
  }
}

template <int IO, int NL>
__device__ __forceinline__ void tx_task_full(const LaunchArgs& a, const TaskDesc& T, const GroupDesc& G, float2* smem,
                             int lmax) {
  float2* S = smem;                    // N-bin spectrum, then the in-place IFFT
  float2* bs = smem + NL;              // short FFT scratch (lmax points)
  float2* pend = bs + lmax;            // OLA carry (N/2)
  const float2* tw = reinterpret_cast<const float2*>(a.twiddle);
  int64_t prev_end = INT64_MIN;
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    const int64_t next_start =
        (T.ola && bi + 1 < T.blk_count) ? a.blk[T.blk_first + bi + 1].t0 : INT64_MAX;
    __syncthreads();
    for (int i = threadIdx.x; i < NL; i += kThreads) S[i] = make_float2(0.f, 0.f);
    for (int m = 0; m < G.n_sb; ++m) {
      const SbDesc Sb = a.sb[G.sb_first + m];
      const BlockSb Z = a.bsb[B.bs + m];
      LoadSeg<IO> ld{a.in, Z.x0, Z.lo, Z.hi};
      StoreAddLong st{S, a.weights + Sb.w_off, make_float2(Z.ph.x, Z.ph.y), Sb.L, NL, Sb.q0};
      __syncthreads();
      switch (Sb.L) {
#define FC_SHORT(LL) case LL: if constexpr (LL <= NL) fft_run<LL, -1>(bs, 0, ld, st, tw); break;
        FC_SHORT(16) FC_SHORT(32) FC_SHORT(64) FC_SHORT(128) FC_SHORT(256) FC_SHORT(512)
        FC_SHORT(1024) FC_SHORT(2048) FC_SHORT(4096)
#undef FC_SHORT
        default: break;
      }
    }
    __syncthreads();
    LoadLds ls{S, 0};
    TxEpi ep;
    ep.pend = pend; ep.t0 = B.t0; ep.prev_end = prev_end;
#pragma unroll
    for (int s = 0; s < 16; ++s) ep.pos[s] = -1;
    fft_run<NL, +1>(S, 0, ls, ep, tw);
    __syncthreads();
    tx_epilogue<IO>(ep, pend, next_start, B.hlo, B.hhi, T, a.out);
    prev_end = T.ola ? B.t0 + NL : INT64_MIN;
  }
}

template <int IO>
__global__ __launch_bounds__(kThreads) void fc_tx_kernel(LaunchArgs a, int lmax) {
  extern __shared__ float2 smem[];
  const int task = blockIdx.x;
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  if (!T.accumulate) {
    zero_range<IO>(a.out, T.z0_lo, T.z0_hi);
    zero_range<IO>(a.out, T.z1_lo, T.z1_hi);
  }
  if (G.prune) {
    switch (a.sb[G.sb_first].L) {
#define FC_PR(LL) case LL: tx_task_pruned<IO, LL>(a, T, G, smem); break;
      FC_PR(16) FC_PR(32) FC_PR(64) FC_PR(128) FC_PR(256) FC_PR(512) FC_PR(1024) FC_PR(2048)
#undef FC_PR
      default: break;
    }
  } else {
    switch (G.N) {
#define FC_FULL(NN) case NN: tx_task_full<IO, NN>(a, T, G, smem, lmax); break;
      FC_FULL(16) FC_FULL(32) FC_FULL(64) FC_FULL(128) FC_FULL(256) FC_FULL(512) FC_FULL(1024)
      FC_FULL(2048) FC_FULL(4096)
#undef FC_FULL
      default: break;
    }
  }
}

// ------------------------------------------------------------- RX tasks ---
template <int IO, int NL>
__device__ __forceinline__ void rx_task(const LaunchArgs& a, const TaskDesc& T, const GroupDesc& G, float2* smem) {
  float2* S = smem;          // long spectrum (N)
  float2* bs = smem + NL;    // short IFFT scratch
  const float2* tw = reinterpret_cast<const float2*>(a.twiddle);
  for (int bi = 0; bi < T.blk_count; ++bi) {
    const BlockDesc B = a.blk[T.blk_first + bi];
    LoadHigh<IO> lh{a.in, B.t0, B.hlo, B.hhi};
    StoreLds sl{S};
    __syncthreads();
    fft_run<NL, -1>(S, 0, lh, sl, tw);
    __syncthreads();
    for (int m = 0; m < G.n_sb; ++m) {
      const SbDesc Sb = a.sb[G.sb_first + m];
      const BlockSb Z = a.bsb[B.bs + m];
      LoadGather lg{S, a.weights + Sb.w_off, make_float2(Z.ph.x, Z.ph.y), Sb.L, NL, Sb.q0};
      StoreLow<IO> so{a.out, Z.x0, Z.lo, Z.hi, T.accumulate != 0};
      switch (Sb.L) {
#define FC_SHORT(LL) case LL: if constexpr (LL <= NL) fft_run<LL, +1>(bs, 0, lg, so, tw); break;
        FC_SHORT(16) FC_SHORT(32) FC_SHORT(64) FC_SHORT(128) FC_SHORT(256) FC_SHORT(512)
        FC_SHORT(1024) FC_SHORT(2048) FC_SHORT(4096)
#undef FC_SHORT
        default: break;
      }
    }
  }
}

template <int IO>
__global__ __launch_bounds__(kThreads) void fc_rx_kernel(LaunchArgs a) {
  extern __shared__ float2 smem[];
  // consecutive tasks (blocks sharing half of their input) go to the same XCD:
  // the dispatcher places workgroup i on XCD i mod 8
  const int n = gridDim.x;
  const int per = (n + 7) >> 3;
  const int x = blockIdx.x & 7, k = blockIdx.x >> 3;
  int task = x * per + k;
  // remap only when the grid is a multiple of 8 (otherwise the map is not a bijection)
  if (n & 7) task = blockIdx.x;
  if (task >= a.n_task) return;
  const TaskDesc T = a.task[task];
  const GroupDesc G = a.grp[T.group];
  switch (G.N) {
#define FC_FULL(NN) case NN: rx_task<IO, NN>(a, T, G, smem); break;
    FC_FULL(16) FC_FULL(32) FC_FULL(64) FC_FULL(128) FC_FULL(256) FC_FULL(512) FC_FULL(1024)
    FC_FULL(2048) FC_FULL(4096)
#undef FC_FULL
    default: break;
  }
}

// ----------------------------------------------------------------- misc ---
template <int IO>
__global__ __launch_bounds__(kThreads) void fc_zero_kernel(void* out, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride)
    st_io<IO>(out, i, make_float2(0.f, 0.f));
}

// ------------------------------------------------------------ launchers ---
hipError_t launch_tx(const LaunchArgs& a, int lmax, size_t lds, hipStream_t s) {
  if (a.n_task <= 0) return hipSuccess;
  dim3 grid(a.n_task), block(kThreads);
  switch (a.io) {
    case IO_C64: hipLaunchKernelGGL(fc_tx_kernel<IO_C64>, grid, block, lds, s, a, lmax); break;
    case IO_F16: hipLaunchKernelGGL(fc_tx_kernel<IO_F16>, grid, block, lds, s, a, lmax); break;
    case IO_BF16: hipLaunchKernelGGL(fc_tx_kernel<IO_BF16>, grid, block, lds, s, a, lmax); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_rx(const LaunchArgs& a, size_t lds, hipStream_t s) {
  if (a.n_task <= 0) return hipSuccess;
  const int n = (a.n_task + 7) & ~7;
  dim3 grid(n), block(kThreads);
  switch (a.io) {
    case IO_C64: hipLaunchKernelGGL(fc_rx_kernel<IO_C64>, grid, block, lds, s, a); break;
    case IO_F16: hipLaunchKernelGGL(fc_rx_kernel<IO_F16>, grid, block, lds, s, a); break;
    case IO_BF16: hipLaunchKernelGGL(fc_rx_kernel<IO_BF16>, grid, block, lds, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_zero(void* out, int64_t n, int io, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kThreads - 1) / kThreads;
  if (blocks > 8192) blocks = 8192;
  dim3 grid((unsigned)blocks), block(kThreads);
  switch (io) {
    case IO_C64: hipLaunchKernelGGL(fc_zero_kernel<IO_C64>, grid, block, 0, s, out, n); break;
    case IO_F16: hipLaunchKernelGGL(fc_zero_kernel<IO_F16>, grid, block, 0, s, out, n); break;
    case IO_BF16: hipLaunchKernelGGL(fc_zero_kernel<IO_BF16>, grid, block, 0, s, out, n); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t set_lds_limits(size_t bytes) {
  hipError_t e = hipSuccess;
  const void* fns[] = {(const void*)fc_tx_kernel<IO_C64>, (const void*)fc_tx_kernel<IO_F16>,
                       (const void*)fc_tx_kernel<IO_BF16>, (const void*)fc_rx_kernel<IO_C64>,
                       (const void*)fc_rx_kernel<IO_F16>, (const void*)fc_rx_kernel<IO_BF16>};
  for (const void* f : fns) {
    hipError_t r = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (r != hipSuccess) e = r;
  }
  return e;
}

}  // namespace fcx

// Host planner and C ABI of the FC library.
//
// The planner turns subband descriptions (Sec. III-A/III-B problem statement)
// into device tables: per-subband constants, processing groups (subbands that
// share a stream, a long transform and a block grid), FC blocks with their
// input/output windows and FP64-computed phases, and tasks (runs of blocks
// processed by one workgroup). All schedule arithmetic is integer; phases are
// evaluated in FP64 from integer-reduced arguments and rounded once to FP32.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "fc.h"
#include "fc_internal.h"

namespace fcx {
hipError_t launch_kernel(int cls, int size, const LaunchArgs& a, int aux, size_t lds, hipStream_t s);
hipError_t launch_zero(void* out, int64_t n, int io, hipStream_t s);
hipError_t set_lds_limits(size_t bytes);
hipError_t noalloc_scratch(int device, float** ptr);
}  // namespace fcx

using namespace fcx;

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }
int64_t imod(int64_t a, int64_t m) { int64_t r = a % m; return r < 0 ? r + m : r; }

// exp(j 2 pi num / den) with the integer argument reduced first, times scale.
Cf unit_phase(int64_t num, int64_t den, double scale) {
  const double ang = 2.0 * kPi * (double)imod(num, den) / (double)den;
  return Cf{(float)(scale * std::cos(ang)), (float)(scale * std::sin(ang))};
}

// Host-side view of one subband.
struct Sub {
  fc_subband d;
  int mu = 0, I = 1, L = 0, N = 0, logL = 0, logN = 0;
  int LO = 0, LS = 0, LL = 0, LT = 0;
  int64_t NO = 0, NS = 0, NL = 0, NT = 0;
  bool sync = false, ola = false;
  std::vector<int> ncp, lcp;   // high- and low-rate CP per symbol
  std::vector<int64_t> pos;    // low-rate start of each symbol in the CP-OFDM stream
  std::vector<int64_t> sig;    // sigma_n: high-rate start of each filtered symbol
  int64_t n_in = 0;            // CP-OFDM stream length (low rate)
  int64_t Q = 0;               // local high-rate span
  int64_t first_cp = 0;        // local high-rate position of the first CP start
  int group = -1;
  int64_t offset = 0;          // position of local sample 0 in the stream
  std::vector<float> w;        // weights (fftshifted)
};

struct Group {
  int stream;
  std::vector<int> subs;       // plan subband indices
  int N;
  bool sync, ola;
  int taper;                   // synchronised OLS TX: output-window edge length
  int64_t offset;              // within the stream
  int64_t Q;
  int rank;                    // order of the group within its stream
  int R;                       // number of blocks
};

// Tables and launch phases of one operation.
struct Op {
  bool valid = false;
  std::vector<int64_t> lo_off;            // n_sb + 1
  std::vector<SbDesc> sb;
  std::vector<GroupDesc> grp;
  std::vector<BlockDesc> blk;
  std::vector<BlockSb> bsb;
  std::vector<TaskDesc> task;
  std::vector<uint64_t> rxmap;            // RX scatter maps
  int64_t part_total = 0;                 // floats of per-task scratch: the weight gradient's partial
                                          // sums, the demodulating RX's second-block terms
  bool part_eager = false;                // scratch allocated with the tables (demodulating RX)
  // One kernel launch. kind: 0 = FC kernel of class cls (0 TX pruned, 1 TX
  // full, 2 RX / adjoint) and transform size `size`; 2 = zero the output
  // buffer. glds: LDS bytes of the weight-gradient kernel over the same tasks
  // (adjoint op only). Consecutive launches with the same seq touch disjoint
  // outputs and may run concurrently; cost is their estimated work.
  struct Phase {
    int kind; int first, count; size_t lds; int aux; int64_t zero_n; int cls, size; size_t glds;
    int seq; double cost;
    int key3;      // third element of the class key (cls, size, key3)
    int tplan;     // transform plan of the launch
  };
  std::vector<Phase> phases;
  // device copies
  SbDesc* d_sb = nullptr; GroupDesc* d_grp = nullptr; BlockDesc* d_blk = nullptr;
  BlockSb* d_bsb = nullptr; TaskDesc* d_task = nullptr;
  uint64_t* d_rxmap = nullptr;
  float* d_part = nullptr;                // per-task scratch (the weight gradient's at its first use)
};

}  // namespace

constexpr int kMaxConc = 4;      // user stream + three side streams
// Internal schedule of the weight gradient: the adjoint's blocks, but tasks of
// a fixed kWgradRun blocks (two synchronised symbols), so that the per-task
// partial sums, added in block order, form the same summation tree for every
// tuning of the adjoint.
constexpr int kOpWgrad = 5;
constexpr int kOps = 6;
constexpr int kWgradRun = 4;

struct fc_plan {
  int device = 0, io = 0;
  std::vector<Sub> subs;
  std::vector<Group> groups;
  int n_streams = 0;
  std::vector<int64_t> hi_off;   // n_streams + 1
  std::vector<int> w_off;        // per subband
  int w_total = 0;
  float* d_w = nullptr;
  Cf* d_tw = nullptr;
  Cf* d_twp = nullptr;           // per-pass twiddle bases
  Op op[kOps];                        // FC_OP_TX .. FC_OP_TXG, then the weight gradient's schedule
  int run_len[5] = {0, 0, 0, 0, 0};   // blocks per task per op (0: planner heuristic)
  int tplan[5] = {0, 0, 0, 0, 0};     // transform plan per op (0 or 1: pruned_ws, rx_long_cap)
  // per-class exceptions to tplan (kernel class key -> plan), chosen by the
  // autotuner; cleared by fc_plan_set_transform_plan
  std::map<std::tuple<int, int, int>, int> class_tp[5];
  int conc[5] = {kMaxConc, kMaxConc, kMaxConc, kMaxConc, kMaxConc};   // per op: launches of one independent set in flight
  hipStream_t side[kMaxConc - 1] = {};
  hipEvent_t ev_fork = nullptr;
  hipEvent_t ev_join[kMaxConc - 1] = {};
};

namespace {

int nr_cp(int N, int mu, int l, int* out) {
  if ((N * 144) % 2048 || ((int64_t)N * (1 << mu) * 16) % 2048) return FC_E_SHAPE;
  int v = N * 144 / 2048;
  if (l % (7 * (1 << mu)) == 0) v += (int)((int64_t)N * (1 << mu) * 16 / 2048);
  *out = v;
  return FC_OK;
}

std::vector<float> rc_default(int L, int K, int ntb) {
  std::vector<float> D(L, 0.f);
  const int h = L / 2;
  for (int k = -K / 2; k < K / 2; ++k) D[h + k] = 1.f;
  for (int i = 1; i <= ntb; ++i) {
    const double w = 0.5 * (1.0 + std::cos(kPi * i / (ntb + 1)));
    D[h + K / 2 - 1 + i] = (float)w;
    D[h - K / 2 - i] = (float)w;
  }
  return D;
}

fc_status analyse(const fc_subband& d, Sub& s) {
  s.d = d;
  s.d.ncp_high = nullptr;
  if (d.n_symbols < 1 || d.n_active < 0 || (d.n_active & 1) || d.n_tb < 0) return FC_E_ARG;
  if (d.mode < FC_CONT_OLA || d.mode > FC_SYNC_OLS || d.stream < 0) return FC_E_ARG;
  if (d.scs_khz <= 0 || d.scs_khz % 15) return FC_E_ARG;
  int ratio = d.scs_khz / 15;
  if (!is_pow2(ratio)) return FC_E_ARG;
  s.mu = ilog2(ratio);
  // powers of two 16..4096 or 3 x 2^k for 768..3072, with n_long / n_short a
  // power of two (the interpolation factor)
  if (!fft_size_ok(d.n_short) || !fft_size_ok(d.n_long)) return FC_E_UNSUPPORTED;
  if (d.n_long < d.n_short) return FC_E_SHAPE;
  if (!divides_pow2(d.n_short, d.n_long)) return FC_E_SHAPE;
  if (d.n_active + 2 * d.n_tb > d.n_short) return FC_E_SHAPE;
  if (std::abs((int64_t)d.center_bin) + d.n_short / 2 > d.n_long / 2) return FC_E_SHAPE;
  if (d.overlap_den <= 0 || d.overlap_num <= 0 || 2 * d.overlap_num > d.overlap_den) return FC_E_UNSUPPORTED;
  s.L = d.n_short; s.N = d.n_long; s.logL = ilog2(s.L); s.logN = ilog2(s.N); s.I = s.N / s.L;
  s.sync = d.mode == FC_SYNC_OLA || d.mode == FC_SYNC_OLS;
  s.ola = d.mode == FC_CONT_OLA || d.mode == FC_SYNC_OLA;
  if (((int64_t)d.overlap_num * s.L) % d.overlap_den) return FC_E_SHAPE;
  s.LO = (int)((int64_t)d.overlap_num * s.L / d.overlap_den);
  if (s.LO & 1) return FC_E_SHAPE;         // N_L = I L_L needs an even split
  if (s.sync && 2 * s.LO != s.L) return FC_E_UNSUPPORTED;
  s.LS = s.L - s.LO; s.LL = (s.LO + 1) / 2; s.LT = s.LO / 2;
  s.NO = (int64_t)s.I * s.LO; s.NS = s.N - s.NO; s.NL = (int64_t)s.I * s.LL; s.NT = (int64_t)s.I * s.LT;
  // CP schedule (Sec. III-A rule or explicit list)
  s.ncp.resize(d.n_symbols);
  s.lcp.resize(d.n_symbols);
  const int per_sf = 14 * (1 << s.mu);
  for (int n = 0; n < d.n_symbols; ++n) {
    int v;
    if (d.ncp_high) {
      v = d.ncp_high[n];
      if (v < 0) return FC_E_ARG;
    } else {
      fc_status st = nr_cp(s.N, s.mu, (d.first_symbol + n) % per_sf, &v);
      if (st) return st;
    }
    s.ncp[n] = v;
    if (!s.sync && v % s.I) return FC_E_SHAPE;      // continuous: integer low-rate CP
    s.lcp[n] = v / s.I;                             // floor (Sec. III-E)
    if (s.sync && (s.lcp[n] > s.LL || 2 * (int64_t)v >= s.N)) return FC_E_SHAPE;
  }
  s.pos.resize(d.n_symbols);
  int64_t p = 0;
  for (int n = 0; n < d.n_symbols; ++n) { s.pos[n] = p; p += s.L + s.lcp[n]; }
  s.n_in = p;
  // sigma_n = n N_OFDM + sum_{q=1..n} N_CP,q (Sec. III-D), N_OFDM = I L_OFDM = N
  s.sig.resize(d.n_symbols);
  int64_t acc = 0;
  for (int n = 0; n < d.n_symbols; ++n) {
    if (n > 0) acc += s.ncp[n];
    s.sig[n] = (int64_t)n * s.N + acc;
  }
  if (s.sync) {
    s.Q = s.NL + s.NT + (int64_t)d.n_symbols * s.N;
    for (int n = 1; n < d.n_symbols; ++n) s.Q += s.ncp[n];
    s.first_cp = s.NL - s.ncp[0];
  } else {
    const int64_t R = (s.n_in + s.LT + s.LS - 1) / s.LS;
    s.Q = (R - 1) * s.NS + s.N;
    s.first_cp = s.NO;
  }
  // smooth output-window edges (synchronised OLS TX): each ramp lies inside
  // the block, next to its kept range
  if (d.taper < 0 || (d.taper & 1) || (d.taper && d.mode != FC_SYNC_OLS)) return FC_E_ARG;
  if (d.taper / 2 > s.NT) return FC_E_SHAPE;
  for (int n = 0; n < d.n_symbols; ++n)
    if (d.taper / 2 > s.NL - s.ncp[n]) return FC_E_SHAPE;
  s.w = rc_default(s.L, d.n_active, d.n_tb);
  return FC_OK;
}

int64_t sigma(const Sub& s, int n) { return s.sig[n]; }

template <class T>
fc_status upload(const std::vector<T>& h, T** d) {
  *d = nullptr;
  if (h.empty()) return FC_OK;
  if (hipMalloc((void**)d, h.size() * sizeof(T)) != hipSuccess) { *d = nullptr; return FC_E_NOMEM; }
  if (hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return FC_E_DEVICE;
  return FC_OK;
}

// Block windows of one subband for one operation.
// kind: 0 TX, 1 RX (paper's receiver of the mode), 2 adjoint of TX,
// 3 synchronised RX with OFDM demodulation (Sec. V-A simplified form).
struct Win { int64_t x0; int lo, hi; };

Win clip_valid(const Sub& s, int64_t xrel, int lo, int hi, int64_t len) {
  // keep local positions i in [lo, hi) with 0 <= xrel + i < len
  int64_t a = std::max<int64_t>(lo, -xrel), b = std::min<int64_t>(hi, len - xrel);
  if (b < a) b = a;
  return Win{xrel, (int)a, (int)b};
}

// Transform plan of the kernel class `key` of op op_index: the autotuner's
// per-class choice where it made one, else the op's plan.
int class_plan(const fc_plan* P, int op_index, const std::tuple<int, int, int>& key) {
  if (op_index >= 5) return 0;
  const auto it = P->class_tp[op_index].find(key);
  return it != P->class_tp[op_index].end() ? it->second : P->tplan[op_index];
}

void build_op(fc_plan* P, int op_index) {
  Op& op = P->op[op_index];
  op = Op();
  // the weight gradient's schedule is the adjoint's, with its own task split
  const bool wgrad = op_index == kOpWgrad;
  const int kind = wgrad ? FC_OP_ADJ : op_index;
  const int nsb = (int)P->subs.size();
  // validity: TX any mode; ADJ CONT_* or SYNC_OLA; RX any; the
  // demodulating RX and the grid-input TX synchronised subbands
  for (const Sub& s : P->subs) {
    if (kind == 2 && s.d.mode == FC_SYNC_OLS) return;
    if ((kind == 3 || kind == 4) && !s.sync) return;
  }
  op.valid = true;
  const int tk = kind == 4 ? 0 : kind;         // the grid-input TX is scheduled as the TX
  // low-rate layout
  op.lo_off.assign(nsb + 1, 0);
  for (int m = 0; m < nsb; ++m) {
    const Sub& s = P->subs[m];
    const int64_t len = kind == 4 ? (int64_t)s.d.n_symbols * s.d.n_active
                        : ((kind == 1 || kind == 3) && s.sync) ? (int64_t)s.d.n_symbols * s.L : s.n_in;
    op.lo_off[m + 1] = op.lo_off[m] + len;
  }
  // processing groups of this operation: the plan's groups, except that an RX
  // group whose subbands exceed what one workgroup holds in LDS is split
  // (each part repeats the long FFT)
  struct OpGroup { int pg; std::vector<int> subs; };
  std::vector<OpGroup> ogroups;
  for (size_t g = 0; g < P->groups.size(); ++g) {
    const Group& G = P->groups[g];
    if (tk == 0) { ogroups.push_back(OpGroup{(int)g, G.subs}); continue; }
    // RX: split so that each part's subband regions fit kRxMaxLds LDS entries
    // and no long bin feeds more than kRxMaxDest of its subbands
    OpGroup cur{(int)g, {}};
    int acc = 0;
    std::vector<int> mult(G.N, 0);
    for (int m : G.subs) {
      const Sub& s = P->subs[m];
      const int q0 = (int)imod((int64_t)s.d.center_bin - s.L / 2, s.N);
      bool over = acc + lds_elems(s.L) > kRxMaxLds;
      for (int p = 0; p < s.L && !over; ++p) over = mult[(q0 + p) % G.N] >= kRxMaxDest;
      if (!cur.subs.empty() && over) {
        ogroups.push_back(cur);
        cur.subs.clear();
        acc = 0;
        std::fill(mult.begin(), mult.end(), 0);
      }
      cur.subs.push_back(m);
      acc += lds_elems(s.L);
      for (int p = 0; p < s.L; ++p) mult[(q0 + p) % G.N]++;
    }
    ogroups.push_back(cur);
  }
  // subband table in group order
  std::unordered_map<uint64_t, int> map_by_hash;     // RX scatter maps by content: group holding it
  for (size_t g = 0; g < ogroups.size(); ++g) {
    const OpGroup& OG = ogroups[g];
    const Group& G = P->groups[OG.pg];
    GroupDesc gd{};
    gd.N = G.N; gd.logN = ilog2(G.N);
    gd.n_sb = (int)OG.subs.size(); gd.sb_first = (int)op.sb.size();
    const Sub& s0 = P->subs[OG.subs[0]];
    // tapered output windows are applied by the full-transform kernel only
    gd.taper = tk == 0 ? G.taper : 0;
    // (mixed-radix sizes always take the full long transform)
    gd.prune = (tk == 0 && OG.subs.size() == 1 && s0.I >= 2 && s0.L >= 16 && !gd.taper && is_pow2(s0.L)) ? 1 : 0;
    op.grp.push_back(gd);
    int cofs = 0;
    for (int m : OG.subs) {
      const Sub& s = P->subs[m];
      SbDesc d{};
      d.L = s.L; d.logL = s.logL; d.c = s.d.center_bin;
      d.q0 = (int)imod((int64_t)s.d.center_bin - s.L / 2, s.N);
      d.w_off = P->w_off[m];
      d.wave = -1;
      d.cofs = cofs;
      cofs += lds_elems(s.L);
      d.lo_off = op.lo_off[m]; d.lo_len = op.lo_off[m + 1] - op.lo_off[m];
      op.sb.push_back(d);
    }
    if (tk != 0) {
      GroupDesc& gr = op.grp.back();
      // scatter map: long bin q feeds IFFT input u = (p + L/2) mod L of every
      // subband with p = (q - q0) mod N < L, at LDS cofs + pad(u)
      gr.map_off = (int)op.rxmap.size();
      op.rxmap.resize(op.rxmap.size() + gr.N, ~0ull);
      std::vector<int> cnt(gr.N, 0);
      for (int i = 0; i < gr.n_sb; ++i) {
        const SbDesc& d = op.sb[gr.sb_first + i];
        for (int pidx = 0; pidx < d.L; ++pidx) {
          const int q = (d.q0 + pidx) % gr.N;
          const int u = (pidx + d.L / 2) % d.L;
          const uint64_t dst = (uint64_t)(d.cofs + u + (u >> 5));
          uint64_t& e = op.rxmap[gr.map_off + q];
          e &= ~(0xffffull << (16 * cnt[q]));
          e |= dst << (16 * cnt[q]);
          cnt[q]++;
        }
        if (d.L > 1024) gr.n_long_sb++;
      }
      // groups with the same subband layout (every frame of a batch of
      // frames) share one copy of the map, so that the copy stays in cache
      // instead of one copy per group streaming through it
      {
        uint64_t hsh = 1469598103934665603ull ^ (uint64_t)gr.N;      // FNV-1a over the entries
        for (int q = 0; q < gr.N; ++q) hsh = (hsh ^ op.rxmap[gr.map_off + q]) * 1099511628211ull;
        auto it = map_by_hash.find(hsh);
        if (it != map_by_hash.end() && op.grp[it->second].N == gr.N &&
            std::equal(op.rxmap.begin() + op.grp[it->second].map_off,
                       op.rxmap.begin() + op.grp[it->second].map_off + gr.N, op.rxmap.begin() + gr.map_off)) {
          op.rxmap.resize(gr.map_off);
          gr.map_off = op.grp[it->second].map_off;
        } else if (it == map_by_hash.end()) {
          map_by_hash[hsh] = (int)g;
        }
      }
      // spread the one-wave short IFFTs (L <= 1024) over the four waves,
      // costliest first onto the least loaded wave. A one-wave transform
      // costs per pass its values per lane plus a fixed overhead (the pass's
      // LDS round trip and wave barrier, about four values' worth): with
      // L log L as the cost the 8-subband filter bank put 512 + 512 + 256
      // points (ten passes) on one wave, and the RX took 1.156 ms against
      // 1.125 ms with this cost
      auto cost = [&](int i) {
        const int Lq = op.sb[i].L;
        if (is_tri(Lq)) {          // three radix-4 sub-transforms of L/3 points, then the combination
          const int P2 = Lq / 3, vsub = ((P2 / 4) + 63) / 64 * 4;
          return (double)3 * npass(P2, 4) * (vsub + 4) + 3 * ((P2 + 63) / 64) + 4;
        }
        const int rm = wave_radix_cap(Lq);
        const int vpl = ((Lq / radix_of(Lq, 0, rm)) + 63) / 64 * radix_of(Lq, 0, rm);
        return (double)npass(Lq, rm) * (vpl + 4);
      };
      std::vector<int> idx;
      for (int i = 0; i < gr.n_sb; ++i)
        if (op.sb[gr.sb_first + i].L <= 1024) idx.push_back(gr.sb_first + i);
      std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return cost(x) > cost(y); });
      double load[4] = {0, 0, 0, 0};
      for (int i : idx) {
        int w = (int)(std::min_element(load, load + 4) - load);
        op.sb[i].wave = w;
        load[w] += cost(i);
      }
      // weight-gradient LDS: spectrum / regions, short-FFT scratch (one per
      // wave, or one workgroup buffer for L > 1024), float accumulators
      int rsum = 0, wmax = 0, lmax_long = 0;
      gr.acc_len = 0;
      for (int i = 0; i < gr.n_sb; ++i) {
        SbDesc& d = op.sb[gr.sb_first + i];
        rsum += lds_elems(d.L);
        if (d.L <= 1024) wmax = std::max(wmax, d.L);
        else lmax_long = std::max(lmax_long, d.L);
        d.aofs = gr.acc_len;
        gr.acc_len += d.L;
      }
      gr.wstride = wmax ? lds_elems(wmax) : 0;
      gr.scr_off = std::max(lds_elems(gr.N), rsum);
      gr.acc_off = gr.scr_off + std::max(4 * gr.wstride, lmax_long ? lds_elems(lmax_long) : 0);
      // one subband with a one-wave short transform: the gradient takes its
      // blocks in groups, one short FFT per wave (instead of one wave busy)
      if (gr.n_sb == 1 && wmax > 0) gr.wg_nb = wgg_group_blocks(wmax, gr.N);
    }
  }
  // blocks and tasks; tasks are collected per launch phase and kernel class
  struct ClassTasks { std::vector<TaskDesc> t; size_t lds = 0; int aux = 0; size_t glds = 0; };
  struct PhaseTasks { std::map<std::tuple<int, int, int>, ClassTasks> cls; };
  std::map<int, PhaseTasks> tx_phase;        // TX: by group rank within the stream
  PhaseTasks rx_all, rx_even, rx_odd;
  bool any_acc_tx = false, any_ola_rx = false;
  int64_t total_blocks = 0;
  for (const Group& o : P->groups) total_blocks += o.sync ? 2 * P->subs[o.subs[0]].d.n_symbols : o.R;
  for (size_t g = 0; g < ogroups.size(); ++g) {
    const OpGroup& OG = ogroups[g];
    const Group& G = P->groups[OG.pg];
    const Sub& s0 = P->subs[OG.subs[0]];
    const int N = G.N;
    const int64_t base = P->hi_off[G.stream] + G.offset;
    const int first_blk = (int)op.blk.size();
    int lmax = 0, lsum = 0;
    for (int m : OG.subs) {
      lmax = std::max(lmax, P->subs[m].L);
      lsum += lds_elems(P->subs[m].L);
    }
    // --- blocks ---
    const int nblk = G.sync ? 2 * s0.d.n_symbols : G.R;
    for (int b = 0; b < nblk; ++b) {
      BlockDesc bd{};
      int64_t t_local;
      const int n = b >> 1, r = G.sync ? (b & 1) : b;
      if (G.sync) t_local = sigma(s0, n) + (int64_t)(b & 1) * (N / 2);
      else t_local = (int64_t)b * s0.NS;
      bd.t0 = base + t_local;
      // high-rate window
      if (tk == 0) {
        if (!G.sync && !G.ola) { bd.hlo = (int)s0.NL; bd.hhi = (int)(s0.NL + s0.NS); }
        else if (G.sync && !G.ola && G.taper) {
          // synchronised OLS with smooth outer edges: the windows overlap at
          // symbol boundaries, so the blocks are combined by OLA; the window
          // itself is applied in the kernel
          const int h = G.taper / 2;
          bd.hlo = 0; bd.hhi = N;
          bd.win = r == 0 ? win_pack((int)(s0.NL - s0.ncp[n]) - h, (int)(s0.NL + s0.NS), true, false)
                          : win_pack((int)s0.NL, (int)(s0.NL + s0.NS) + h, false, true);
        } else if (G.sync && !G.ola) {
          // synchronised OLS: the synthesis windows s_0 (from the CP start) and s_1
          bd.hlo = r == 0 ? (int)(s0.NL - s0.ncp[n]) : (int)s0.NL;
          bd.hhi = (int)(s0.NL + s0.NS);
        } else { bd.hlo = 0; bd.hhi = N; }
      } else {
        // RX of CONT_OLA (G^(OLA)) and ADJ of CONT_OLS window the high-rate input
        const bool win = !G.sync && ((kind == 1 && G.ola) || (kind == 2 && !G.ola));
        if (win) { bd.hlo = (int)s0.NL; bd.hhi = (int)(s0.NL + s0.NS); }
        else { bd.hlo = 0; bd.hhi = N; }
      }
      bd.bs = (int)op.bsb.size();
      op.blk.push_back(bd);
      for (int m : OG.subs) {
        const Sub& s = P->subs[m];
        const int L = s.L;
        BlockSb z{};
        Win w{};
        int64_t phase_num;       // exponent of exp(j 2 pi phase_num / N)
        if (G.sync) {
          const int S_L = s.LL - s.lcp[n];
          phase_num = (int64_t)r * s.d.center_bin * (N / 2) + (int64_t)s.d.center_bin * sigma(s, n);
          if (kind == 1) {
            // Sec. IV concatenation: keep [L/4, 3L/4) of both blocks, CP removed
            const int64_t xrel = (int64_t)n * L + (int64_t)r * (L / 2) - L / 4;
            w = Win{xrel, L / 4, 3 * L / 4};
          } else if (kind == 3) {
            // the symbol's L subcarriers, written when its second block is done
            w = Win{(int64_t)n * L, 0, L};
          } else {
            const int64_t xrel = s.pos[n] + (int64_t)r * (L / 2) - S_L;
            if (G.ola)       // OLA analysis windows a_0, a_1
              w = (r == 0) ? Win{xrel, S_L, 3 * L / 4} : Win{xrel, L / 4, 3 * L / 4};
            else             // OLS: the whole block of z = [0_{S_L}; x_CP; 0_{L_T}]
              w = (r == 0) ? Win{xrel, S_L, L} : Win{xrel, 0, 3 * L / 4};
          }
        } else {
          phase_num = (int64_t)r * s.d.center_bin * s.LS * s.I;   // r c L_S / L in units of 1/N
          const int64_t xrel = (int64_t)r * s.LS - s.LO;
          bool low_window;      // TX input window a / RX keep window a, else full block
          if (tk == 0) low_window = G.ola;
          else if (kind == 1) low_window = !G.ola;           // G^(OLS) keeps [L_L, L_L + L_S)
          else low_window = G.ola;                           // adjoint of TX-OLA: keep a
          w = low_window ? clip_valid(s, xrel, s.LL, s.LL + s.LS, s.n_in)
                         : clip_valid(s, xrel, 0, L, s.n_in);
        }
        z.x0 = op.lo_off[m] + w.x0;
        z.lo = w.lo; z.hi = w.hi;
        if (kind == 4) {
          // block sample i of z = [0_{S_L}; x_CP; 0_{L_T}] at r L/2 is OFDM sample
          // (r L/2 + i - L/4) mod L of the symbol (S_L + L_CP,n = L/4)
          z.x0 = op.lo_off[m] + (int64_t)n * s.d.n_active;
          z.shift = r ? L / 4 : 3 * L / 4;
          z.K = s.d.n_active;
        }
        if (tk == 0) z.ph = unit_phase(phase_num, N, std::sqrt((double)s.I) / N);
        else if (kind == 3) z.ph = unit_phase(-phase_num, N, 1.0 / std::sqrt((double)s.I));   // g^(r) itself
        else z.ph = unit_phase(-phase_num, N, 1.0 / (std::sqrt((double)s.I) * L));
        op.bsb.push_back(z);
      }
    }
    const int64_t span_lo = base, span_hi = base + G.Q;
    if (tk == 0) {
      // --- TX runs ---
      const bool acc = P->groups.size() > 1 &&
          std::count_if(P->groups.begin(), P->groups.end(), [&](const Group& o) { return o.stream == G.stream; }) > 1;
      any_acc_tx |= acc;
      const bool ola = G.ola || G.taper > 0;
      int K = P->run_len[0] > 0 ? P->run_len[0]
                                : (int)std::max<int64_t>(8, std::min<int64_t>(64, total_blocks / 2048));
      if (G.sync) K += K & 1;                           // whole symbols per run
      for (int b0 = 0; b0 < nblk; b0 += K) {
        const int b1 = std::min(nblk, b0 + K);
        TaskDesc t{};
        t.group = (int)g;
        t.ola = ola ? 1 : 0;
        t.accumulate = acc ? 1 : 0;
        t.warm = (ola && b0 > 0) ? 1 : 0;
        t.blk_first = first_blk + b0 - t.warm;
        t.blk_count = b1 - b0 + t.warm;
        const BlockDesc& B0 = op.blk[first_blk + b0];
        const BlockDesc& Bl = op.blk[first_blk + b1 - 1];
        if (ola) {
          t.own_lo = (b0 == 0) ? span_lo : B0.t0;
          t.own_hi = (b1 == nblk) ? span_hi : op.blk[first_blk + b1].t0;
        } else {
          t.own_lo = (b0 == 0) ? span_lo : B0.t0 + B0.hlo;
          t.own_hi = (b1 == nblk) ? span_hi : Bl.t0 + Bl.hhi;
          if (!acc) {
            if (b0 == 0) { t.z0_lo = span_lo; t.z0_hi = B0.t0 + B0.hlo; }
            if (b1 == nblk) { t.z1_lo = Bl.t0 + Bl.hhi; t.z1_hi = span_hi; }
          }
        }
        const GroupDesc& gd = op.grp[g];
        const std::tuple<int, int, int> key =
            gd.prune ? std::make_tuple(0, s0.L, ilog2(s0.I)) : std::make_tuple(1, N, 0);
        ClassTasks& ct = tx_phase[G.rank].cls[key];
        ct.t.push_back(t);
        if (gd.prune) {
          ct.aux = ilog2(s0.I);
          // long IFFT buffer, OLA carry, and (L <= 1024) the short-FFT / band regions
          ct.lds = std::max(ct.lds, (size_t)pruned_lds_bytes(s0.L, N, class_plan(P, op_index, key)));
        } else {
          ct.aux = std::max(ct.aux, lmax);
          ct.lds = std::max(ct.lds, (size_t)(lds_elems(N) + lds_elems(ct.aux) + N / 2) * 8);
        }
      }
    } else {
      // --- RX tasks: runs of consecutive blocks (the next block's input is
      // prefetched while the current one is analysed); in accumulate mode
      // single blocks, split into even and odd launches so no two tasks of a
      // launch add into the same low-rate samples ---
      // (the gradient writes no low-rate samples: it never accumulates)
      const bool acc = !wgrad && !G.sync && ((kind == 1 && G.ola) || (kind == 2 && !G.ola));
      any_ola_rx |= acc;
      int K = wgrad ? kWgradRun
              : acc ? 1
                    : P->run_len[kind] > 0 ? P->run_len[kind]
                                           : (int)std::max<int64_t>(2, std::min<int64_t>(8, total_blocks / 4096));
      if (kind == 3) K += K & 1;                        // whole symbols per task
      // per-task scratch slots, in block order: the weight gradient's partial
      // sums (one float per weight), the demodulating RX's second-block terms
      // (one complex value per subband bin)
      GroupDesc& gw = op.grp[g];
      // demodulating RX: the second-block terms in a second LDS region set
      // where that keeps the kernel's occupancy, else in device scratch
      const size_t lds_one = (size_t)std::max(lds_elems(N), lsum) * 8;
      const bool gb = kind == 3 && !rxd_terms_in_lds(P->io, (int)(lds_one + (size_t)lsum * 8));
      const int64_t slot = wgrad ? gw.acc_len : gb ? 2 * (int64_t)gw.acc_len : 0;
      gw.part_base = op.part_total;
      gw.part_n = (nblk + K - 1) / K;
      op.part_total += (int64_t)gw.part_n * slot;
      op.part_eager = kind == 3 && !wgrad;
      for (int b = 0; b < nblk; b += K) {
        TaskDesc t{};
        t.group = (int)g; t.blk_first = first_blk + b; t.blk_count = std::min(K, nblk - b);
        t.accumulate = acc ? 1 : 0;
        t.part_off = gw.part_base + (int64_t)(b / K) * slot;
        PhaseTasks& ph = acc ? ((b & 1) ? rx_odd : rx_even) : rx_all;
        const GroupDesc& gd = op.grp[g];
        // adjoint: one-subband groups with a whole-workgroup short transform
        // get launches of their own, whose weight gradient keeps its sums in
        // registers (no LDS accumulators: one more workgroup per CU)
        const bool greg = kind == 2 && gd.n_sb == 1 && gd.n_long_sb == 1;
        ClassTasks& ct = ph.cls[std::make_tuple(kind == 3 ? 4 : 2, N, (greg || gb) ? 1 : 0)];
        ct.t.push_back(t);
        ct.aux = gb ? 1 : 0;
        ct.lds = std::max(ct.lds, kind == 3 && !gb ? lds_one + (size_t)lsum * 8 : lds_one);
        ct.glds = std::max(ct.glds, gd.wg_nb ? (size_t)wgg_lds_entries(lmax, N, gd.wg_nb) * 8
                                    : greg   ? (size_t)gd.acc_off * 8
                                             : (size_t)(gd.acc_off + (gd.acc_len + 1) / 2) * 8);
      }
    }
  }
  auto emit = [&](PhaseTasks& ph, bool sort_cost, int seq) {
    // largest transforms first (several launches of one phase are independent)
    std::vector<std::pair<std::tuple<int, int, int>, ClassTasks*>> order;
    for (auto& kv : ph.cls) order.push_back({kv.first, &kv.second});
    // largest transforms first: long size = size << log2 I for pruned classes
    auto work = [](const std::tuple<int, int, int>& k) {
      return std::get<0>(k) == 0 ? std::get<1>(k) << std::get<2>(k) : std::get<1>(k);
    };
    std::stable_sort(order.begin(), order.end(), [&](const auto& a, const auto& b) {
      return work(a.first) > work(b.first);
    });
    for (auto& kv : order) {
      ClassTasks& ct = *kv.second;
      if (ct.t.empty()) continue;
      if (sort_cost) {
        // heavier tasks first: the dispatcher hands workgroups out in index order
        std::stable_sort(ct.t.begin(), ct.t.end(), [&](const TaskDesc& a, const TaskDesc& b) {
          auto cost = [&](const TaskDesc& t) { return (int64_t)op.grp[t.group].N * t.blk_count; };
          return cost(a) > cost(b);
        });
      }
      double cost = 0;
      for (const TaskDesc& t : ct.t) cost += (double)op.grp[t.group].N * t.blk_count;
      Op::Phase p{0, (int)op.task.size(), (int)ct.t.size(), ct.lds, ct.aux, 0, std::get<0>(kv.first),
                  std::get<1>(kv.first), ct.glds, seq, cost, std::get<2>(kv.first),
                  class_plan(P, op_index, kv.first)};
      op.task.insert(op.task.end(), ct.t.begin(), ct.t.end());
      op.phases.push_back(p);
    }
  };
  if (tk == 0) {
    if (any_acc_tx) op.phases.push_back(Op::Phase{2, 0, 0, 0, 0, P->hi_off.back(), 0, 0, 0, -1, 0});
    // groups of one rank belong to different streams: their launches are independent
    for (auto& kv : tx_phase) emit(kv.second, true, kv.first);
  } else {
    if (any_ola_rx) op.phases.push_back(Op::Phase{2, 0, 0, 0, 0, op.lo_off.back(), 0, 0, 0, -1, 0});
    // RX tasks keep block order (neighbouring blocks share input in L2).
    // Accumulating tasks: even blocks, then odd ones (they share samples).
    emit(rx_all, false, 0);
    emit(rx_even, false, 0);
    emit(rx_odd, false, 1);
  }
}

fc_status upload_op(Op& op) {
  if (!op.valid) return FC_OK;
  fc_status s;
  if ((s = upload(op.sb, &op.d_sb))) return s;
  if ((s = upload(op.grp, &op.d_grp))) return s;
  if ((s = upload(op.blk, &op.d_blk))) return s;
  if ((s = upload(op.bsb, &op.d_bsb))) return s;
  if ((s = upload(op.task, &op.d_task))) return s;
  if ((s = upload(op.rxmap, &op.d_rxmap))) return s;
  if (op.part_eager && op.part_total > 0 &&
      hipMalloc((void**)&op.d_part, (size_t)op.part_total * sizeof(float)) != hipSuccess) {
    op.d_part = nullptr;
    return FC_E_NOMEM;
  }
  return FC_OK;
}

void free_op(Op& op) {
  (void)hipFree(op.d_sb); (void)hipFree(op.d_grp); (void)hipFree(op.d_blk); (void)hipFree(op.d_bsb); (void)hipFree(op.d_task);
  (void)hipFree(op.d_rxmap);
  (void)hipFree(op.d_part);
  op.d_rxmap = nullptr;
  op.d_part = nullptr;
  op.d_sb = nullptr; op.d_grp = nullptr; op.d_blk = nullptr; op.d_bsb = nullptr; op.d_task = nullptr;
}

hipError_t launch_phase(fc_plan* P, const Op& op, const Op::Phase& ph, const void* in, void* out, hipStream_t st) {
  if (ph.kind == 2) return launch_zero(out, ph.zero_n, P->io, st);
  LaunchArgs a{};
  a.sb = op.d_sb; a.grp = op.d_grp; a.blk = op.d_blk; a.bsb = op.d_bsb;
  a.task = op.d_task + ph.first; a.n_task = ph.count; a.io = P->io;
  a.weights = P->d_w; a.twiddle = P->d_tw; a.twpass = P->d_twp; a.rxmap = op.d_rxmap;
  a.in = in; a.out = out; a.part = op.d_part;
  a.front = &op == &P->op[FC_OP_TXG] ? 1 : 0;
  a.tplan = ph.tplan;
  return launch_kernel(ph.cls, ph.size, a, ph.aux, ph.lds, st);
}

// Launches the op's phases in order. A run of phases with one seq is
// independent work: it is spread over the caller's stream and up to
// conc - 1 side streams (fork and join through events, so the caller's
// stream order is kept and a graph capture of the caller's stream records
// the branches).
fc_status run_op(fc_plan* P, int kind, const void* in, void* out, hipStream_t st) {
  Op& op = P->op[kind];
  if (!op.valid || P->device < 0) return FC_E_STATE;
  if (!in || !out) return FC_E_ARG;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  hipError_t e = hipSuccess;
  const size_t n = op.phases.size();
  for (size_t i = 0; i < n && e == hipSuccess;) {
    size_t j = i + 1;
    while (j < n && op.phases[j].kind != 2 && op.phases[i].kind != 2 && op.phases[j].seq == op.phases[i].seq) ++j;
    const int ways = std::min<int>(P->conc[kind], (int)(j - i));
    if (ways <= 1) {
      for (size_t k = i; k < j && e == hipSuccess; ++k) e = launch_phase(P, op, op.phases[k], in, out, st);
    } else {
      e = hipEventRecord(P->ev_fork, st);
      for (int q = 0; q + 1 < ways && e == hipSuccess; ++q) e = hipStreamWaitEvent(P->side[q], P->ev_fork, 0);
      double load[kMaxConc] = {};
      for (size_t k = i; k < j && e == hipSuccess; ++k) {
        const int q = (int)(std::min_element(load, load + ways) - load);
        load[q] += op.phases[k].cost;
        e = launch_phase(P, op, op.phases[k], in, out, q == 0 ? st : P->side[q - 1]);
      }
      for (int q = 0; q + 1 < ways && e == hipSuccess; ++q) {
        e = hipEventRecord(P->ev_join[q], P->side[q]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, P->ev_join[q], 0);
      }
    }
    i = j;
  }
  if (cur != P->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? FC_OK : FC_E_DEVICE;
}

// Weight gradient: the gradient kernel over the adjoint's tasks (its blocks
// carry the forward windows and the adjoint phases), each task storing its
// per-bin sums in its own slot of `part` (the adjoint op's part_total floats),
// then the reduction, which writes every weight of grad_w.
fc_status launch_wgrad(fc_plan* P, const void* x, const void* g, float* grad_w, float* part, hipStream_t st) {
  const Op& op = P->op[kOpWgrad];
  auto launch = [&](const Op::Phase& ph, hipStream_t s) {
    LaunchArgs a{};
    a.sb = op.d_sb; a.grp = op.d_grp; a.blk = op.d_blk; a.bsb = op.d_bsb;
    a.task = op.d_task + ph.first; a.n_task = ph.count; a.io = P->io;
    a.weights = P->d_w; a.twiddle = P->d_tw; a.twpass = P->d_twp; a.rxmap = op.d_rxmap;
    a.in = g; a.out = grad_w; a.in2 = x; a.part = part;
    return launch_kernel(3, ph.size, a, ph.aux, ph.glds, s);
  };
  // the adjoint's independent launch sets, spread over the side streams as
  // run_op does (every task writes only its own slot)
  std::vector<const Op::Phase*> ph;
  for (const Op::Phase& p : op.phases)
    if (p.kind != 2) ph.push_back(&p);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < ph.size() && e == hipSuccess;) {
    size_t j = i + 1;
    while (j < ph.size() && ph[j]->seq == ph[i]->seq) ++j;
    const int ways = std::min<int>(P->conc[FC_OP_ADJ], (int)(j - i));
    if (ways <= 1) {
      for (size_t k = i; k < j && e == hipSuccess; ++k) e = launch(*ph[k], st);
    } else {
      e = hipEventRecord(P->ev_fork, st);
      for (int q = 0; q + 1 < ways && e == hipSuccess; ++q) e = hipStreamWaitEvent(P->side[q], P->ev_fork, 0);
      double load[kMaxConc] = {};
      for (size_t k = i; k < j && e == hipSuccess; ++k) {
        const int q = (int)(std::min_element(load, load + ways) - load);
        load[q] += ph[k]->cost;
        e = launch(*ph[k], q == 0 ? st : P->side[q - 1]);
      }
      for (int q = 0; q + 1 < ways && e == hipSuccess; ++q) {
        e = hipEventRecord(P->ev_join[q], P->side[q]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, P->ev_join[q], 0);
      }
    }
    i = j;
  }
  if (e == hipSuccess) {
    LaunchArgs a{};
    a.sb = op.d_sb; a.grp = op.d_grp; a.n_task = (int)op.grp.size(); a.io = P->io;
    a.out = grad_w; a.part = part;
    e = launch_kernel(5, 0, a, 0, 0, st);
  }
  return e == hipSuccess ? FC_OK : FC_E_DEVICE;
}

fc_status run_wgrad(fc_plan* P, const void* x, const void* g, float* grad_w, hipStream_t st) {
  Op& op = P->op[kOpWgrad];
  if (!op.valid || P->device < 0) return FC_E_STATE;
  if (!x || !g || !grad_w) return FC_E_ARG;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  fc_status r = FC_OK;
  // the partial sums live in plan-owned scratch, allocated at the first call
  // after the adjoint's tasks were (re)built; not while the stream is being
  // captured into a graph (an allocation there would fail the capture)
  if (!op.d_part) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess) r = FC_E_DEVICE;
    else if (cs != hipStreamCaptureStatusNone) r = FC_E_STATE;
    else if (hipMalloc((void**)&op.d_part, (size_t)op.part_total * sizeof(float)) != hipSuccess) {
      op.d_part = nullptr;
      r = FC_E_NOMEM;
    }
  }
  if (r == FC_OK) r = launch_wgrad(P, x, g, grad_w, op.d_part, st);
  if (cur != P->device) (void)hipSetDevice(cur);
  return r;
}

// Measured schedule: times every kernel launch of the op on its own (one
// warm-up, minimum of two), stores the times as the launches' costs and
// orders each independent set by decreasing cost, so that run_op's greedy
// spread over the streams is the longest-processing-time-first rule on
// measured rather than estimated work.
fc_status measure_costs(fc_plan* P, int kind, const void* in, void* out, hipStream_t st, hipEvent_t e0,
                        hipEvent_t e1) {
  Op& op = P->op[kind];
  for (Op::Phase& ph : op.phases) {
    if (ph.kind == 2) continue;
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      if (hipEventRecord(e0, st) != hipSuccess || launch_phase(P, op, ph, in, out, st) != hipSuccess ||
          hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
        return FC_E_DEVICE;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return FC_E_DEVICE;
      if (rep > 0) best = std::min(best, ms);
    }
    ph.cost = best;
  }
  for (size_t i = 0; i < op.phases.size();) {
    size_t j = i + 1;
    while (j < op.phases.size() && op.phases[j].kind != 2 && op.phases[i].kind != 2 &&
           op.phases[j].seq == op.phases[i].seq)
      ++j;
    std::stable_sort(op.phases.begin() + i, op.phases.begin() + j,
                     [](const Op::Phase& a, const Op::Phase& b) { return a.cost > b.cost; });
    i = j;
  }
  return FC_OK;
}

// Dynamic LDS beyond 64 KiB must be granted per kernel function before the
// plan's launches (the grant is process-wide and only ever raised).
fc_status grant_lds(const fc_plan* P) {
  size_t lds_max = 0;
  for (int k = 0; k < kOps; ++k)
    for (const auto& ph : P->op[k].phases) lds_max = std::max(lds_max, std::max(ph.lds, ph.glds));
  if (lds_max > 65536 && set_lds_limits(lds_max) != hipSuccess) return FC_E_UNSUPPORTED;
  return FC_OK;
}

// Rebuild one op's tables with the plan's current tuning (device work on the
// old tables must have finished).
fc_status rebuild_op(fc_plan* P, int kind) {
  if (P->device >= 0) free_op(P->op[kind]);
  build_op(P, kind);
  if (P->device < 0) return FC_OK;
  const fc_status st = upload_op(P->op[kind]);
  return st ? st : grant_lds(P);
}

}  // namespace

// ===================================================================== ABI ==
extern "C" {

const char* fc_status_str(fc_status s) {
  switch (s) {
    case FC_OK: return "ok";
    case FC_E_ARG: return "invalid argument";
    case FC_E_SHAPE: return "inconsistent sizes";
    case FC_E_UNSUPPORTED: return "unsupported configuration";
    case FC_E_NOMEM: return "out of memory";
    case FC_E_DEVICE: return "HIP runtime error";
    case FC_E_STATE: return "operation not valid for this plan";
    case FC_E_LIMIT: return "needs more than the fixed no-allocation scratch";
    default: return "unknown status";
  }
}

const char* fc_version(void) { return "fc 0.1 gfx950"; }

fc_status fc_plan_create(const fc_subband* sb, int32_t n_sb, int32_t io_type, int32_t device, fc_plan** plan) {
  if (!plan) return FC_E_ARG;
  *plan = nullptr;
  if (!sb || n_sb <= 0 || io_type < FC_IO_C64 || io_type > FC_IO_BF16 || device < -1) return FC_E_ARG;
  fc_plan* P = new (std::nothrow) fc_plan();
  if (!P) return FC_E_NOMEM;
  P->device = device;
  P->io = io_type;
  P->subs.resize(n_sb);
  int max_stream = -1;
  for (int m = 0; m < n_sb; ++m) {
    fc_status s = analyse(sb[m], P->subs[m]);
    if (s) { delete P; return s; }
    max_stream = std::max(max_stream, sb[m].stream);
  }
  P->n_streams = max_stream + 1;
  std::vector<int> used(P->n_streams, 0);
  for (int m = 0; m < n_sb; ++m) used[sb[m].stream] = 1;
  for (int u : used) if (!u) { delete P; return FC_E_ARG; }
  // processing groups: same stream, long transform, model and CP schedule
  std::map<std::tuple<int, int, int, int, int, std::vector<int>, int>, int> key2g;
  for (int m = 0; m < n_sb; ++m) {
    Sub& s = P->subs[m];
    auto key = std::make_tuple(s.d.stream, s.N, s.d.mode, s.d.overlap_num * 4096 / s.d.overlap_den,
                               s.d.n_symbols, s.ncp, s.d.taper);
    auto it = key2g.find(key);
    if (it == key2g.end()) {
      Group g{};
      g.stream = s.d.stream; g.N = s.N; g.sync = s.sync; g.ola = s.ola; g.taper = s.d.taper;
      g.Q = s.Q;
      g.R = s.sync ? 2 * s.d.n_symbols : (int)((s.n_in + s.LT + s.LS - 1) / s.LS);
      key2g[key] = (int)P->groups.size();
      P->groups.push_back(g);
      it = key2g.find(key);
    }
    Group& g = P->groups[it->second];
    if (g.Q != s.Q) { delete P; return FC_E_SHAPE; }
    g.subs.push_back(m);
    s.group = it->second;
  }
  // align the groups of each stream on their first CP start; stream lengths
  std::vector<int64_t> len(P->n_streams, 0), tmax(P->n_streams, INT64_MIN);
  std::vector<int> rank(P->n_streams, 0);
  for (Group& g : P->groups) {
    const Sub& s = P->subs[g.subs[0]];
    tmax[g.stream] = std::max(tmax[g.stream], s.first_cp);
    g.rank = rank[g.stream]++;
  }
  for (Group& g : P->groups) {
    const Sub& s = P->subs[g.subs[0]];
    g.offset = tmax[g.stream] - s.first_cp;
    len[g.stream] = std::max(len[g.stream], g.offset + g.Q);
    for (int m : g.subs) P->subs[m].offset = g.offset;
  }
  P->hi_off.assign(P->n_streams + 1, 0);
  for (int k = 0; k < P->n_streams; ++k) P->hi_off[k + 1] = P->hi_off[k] + len[k];
  // weights
  P->w_off.resize(n_sb);
  for (int m = 0; m < n_sb; ++m) { P->w_off[m] = P->w_total; P->w_total += P->subs[m].L; }
  // host tables
  for (int k = 0; k < kOps; ++k) build_op(P, k);
  if (device < 0) {        // host-only plan: schedules and layouts, no device state
    *plan = P;
    return FC_OK;
  }
  // device state
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) { delete P; return FC_E_DEVICE; }
  if (hipSetDevice(device) != hipSuccess) { delete P; return FC_E_DEVICE; }
  fc_status st = FC_OK;
  std::vector<Cf> tw(kTwiddleN);
  for (int k = 0; k < kTwiddleN; ++k) {
    const double a = 2.0 * kPi * k / kTwiddleN;
    tw[k] = Cf{(float)std::cos(a), (float)-std::sin(a)};
  }
  // per-pass bases w^1, w^2, w^4, w^8 of w = exp(-j 2 pi k / (NS R)) for every
  // non-first pass of every transform size and radix plan (layout: twb_off)
  std::vector<Cf> twp(twb_total() + kTw3N);
  for (int RM : {16, 8, 4}) {
    for (int Pn = 2; Pn <= kMaxPoints; Pn <<= 1) {
      for (int sp = 1; sp < npass(Pn, RM); ++sp) {
        const int NS = ns_of(Pn, sp, RM), R = radix_of(Pn, sp, RM);
        for (int k = 0; k < NS; ++k) {
          const int e[4] = {1, 2, 4, 8};
          for (int q = 0; q < 4; ++q) {
            const int64_t num = imod((int64_t)k * e[q], (int64_t)NS * R);
            const double a = 2.0 * kPi * (double)num / (double)(NS * R);
            twp[twb_off(Pn, sp, RM) + 4 * k + q] = Cf{(float)std::cos(a), (float)-std::sin(a)};
          }
        }
      }
    }
  }
  // radix-3 combination of the mixed-radix sizes: exp(-j 2 pi k / 3072)
  for (int k = 0; k < kTw3N; ++k) {
    const double a = 2.0 * kPi * k / kTw3N;
    twp[twb_total() + k] = Cf{(float)std::cos(a), (float)-std::sin(a)};
  }
  std::vector<float> w(P->w_total);
  for (int m = 0; m < n_sb; ++m) std::copy(P->subs[m].w.begin(), P->subs[m].w.end(), w.begin() + P->w_off[m]);
  if (!st) st = upload(tw, &P->d_tw);
  if (!st) st = upload(twp, &P->d_twp);
  if (!st) st = upload(w, &P->d_w);
  for (int k = 0; k < kOps && !st; ++k) st = upload_op(P->op[k]);
  if (!st) st = grant_lds(P);
  // side streams (default priority) and fork/join events
  for (int q = 0; q + 1 < kMaxConc && !st; ++q) {
    if (hipStreamCreateWithFlags(&P->side[q], hipStreamNonBlocking) != hipSuccess) { P->side[q] = nullptr; st = FC_E_DEVICE; }
    else if (hipEventCreateWithFlags(&P->ev_join[q], hipEventDisableTiming) != hipSuccess) { P->ev_join[q] = nullptr; st = FC_E_DEVICE; }
  }
  if (!st && hipEventCreateWithFlags(&P->ev_fork, hipEventDisableTiming) != hipSuccess) { P->ev_fork = nullptr; st = FC_E_DEVICE; }
  (void)hipSetDevice(cur);
  if (st) { fc_plan_destroy(P); return st; }
  *plan = P;
  return FC_OK;
}

void fc_plan_destroy(fc_plan* P) {
  if (!P) return;
  if (P->device < 0) { delete P; return; }
  int cur = -1;
  (void)hipGetDevice(&cur);
  (void)hipSetDevice(P->device);
  for (int q = 0; q + 1 < kMaxConc; ++q) {
    if (P->side[q]) { (void)hipStreamSynchronize(P->side[q]); (void)hipStreamDestroy(P->side[q]); }
    if (P->ev_join[q]) (void)hipEventDestroy(P->ev_join[q]);
  }
  if (P->ev_fork) (void)hipEventDestroy(P->ev_fork);
  for (int k = 0; k < kOps; ++k) free_op(P->op[k]);
  (void)hipFree(P->d_w);
  (void)hipFree(P->d_tw);
  (void)hipFree(P->d_twp);
  if (cur >= 0) (void)hipSetDevice(cur);
  delete P;
}

fc_status fc_plan_counts(const fc_plan* P, int32_t* n_sb, int32_t* n_streams) {
  if (!P) return FC_E_ARG;
  if (n_sb) *n_sb = (int32_t)P->subs.size();
  if (n_streams) *n_streams = P->n_streams;
  return FC_OK;
}

fc_status fc_plan_layout(const fc_plan* P, int32_t op, int64_t* lowrate_off, int64_t* highrate_off) {
  if (!P || op < FC_OP_TX || op > FC_OP_TXG) return FC_E_ARG;
  const Op& o = P->op[op];
  if (!o.valid) return FC_E_STATE;
  if (lowrate_off) std::copy(o.lo_off.begin(), o.lo_off.end(), lowrate_off);
  if (highrate_off) std::copy(P->hi_off.begin(), P->hi_off.end(), highrate_off);
  return FC_OK;
}

fc_status fc_plan_symbols(const fc_plan* P, int32_t sb, int32_t* ncp_high, int32_t* ncp_low, int64_t* offset) {
  if (!P || sb < 0 || sb >= (int)P->subs.size()) return FC_E_ARG;
  const Sub& s = P->subs[sb];
  if (ncp_high) std::copy(s.ncp.begin(), s.ncp.end(), ncp_high);
  if (ncp_low) std::copy(s.lcp.begin(), s.lcp.end(), ncp_low);
  if (offset) *offset = s.offset;
  return FC_OK;
}

fc_status fc_set_weights(fc_plan* P, int32_t sb, const float* w_host, int32_t n, void* stream) {
  if (!P || !w_host || sb < 0 || sb >= (int)P->subs.size()) return FC_E_ARG;
  Sub& s = P->subs[sb];
  if (n != s.L) return FC_E_SHAPE;
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(w_host[i])) return FC_E_ARG;
  std::copy(w_host, w_host + n, s.w.begin());
  if (P->device < 0) return FC_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  hipError_t e = hipMemcpyAsync(P->d_w + P->w_off[sb], s.w.data(), n * sizeof(float), hipMemcpyHostToDevice,
                                (hipStream_t)stream);
  // the plan's host copy is rewritten by the next call: wait for this copy
  if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
  if (cur != P->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? FC_OK : FC_E_DEVICE;
}

fc_status fc_set_weights_device(fc_plan* P, int32_t sb, const float* w_dev, int32_t n, void* stream) {
  if (!P || !w_dev || sb < -1 || sb >= (int)P->subs.size()) return FC_E_ARG;
  if (P->device < 0) return FC_E_STATE;
  // sb == -1: every subband's weights, concatenated in plan order
  if (n != (sb < 0 ? P->w_total : P->subs[sb].L)) return FC_E_SHAPE;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  hipError_t e = hipMemcpyAsync(P->d_w + (sb < 0 ? 0 : P->w_off[sb]), w_dev, n * sizeof(float),
                                hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (cur != P->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? FC_OK : FC_E_DEVICE;
}

fc_status fc_get_weights(const fc_plan* P, int32_t sb, float* w_host, int32_t n) {
  if (!P || !w_host || sb < 0 || sb >= (int)P->subs.size()) return FC_E_ARG;
  const Sub& s = P->subs[sb];
  if (n != s.L) return FC_E_SHAPE;
  if (P->device < 0) {
    std::copy(s.w.begin(), s.w.end(), w_host);
    return FC_OK;
  }
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(w_host, P->d_w + P->w_off[sb], n * sizeof(float), hipMemcpyDeviceToHost);
  if (cur != P->device) (void)hipSetDevice(cur);
  return e == hipSuccess ? FC_OK : FC_E_DEVICE;
}

fc_status fc_plan_set_tuning(fc_plan* P, int32_t op, int32_t run_len, int32_t conc) {
  if (!P || op < 0 || op > 4 || run_len < 0 || run_len > 256 || conc < 1 || conc > kMaxConc) return FC_E_ARG;
  if (!P->op[op].valid) return FC_E_STATE;
  if (P->device >= 0) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    P->run_len[op] = run_len;
    P->conc[op] = conc;
    const fc_status st = ok ? rebuild_op(P, op) : FC_E_DEVICE;
    (void)hipSetDevice(cur);
    return st;
  }
  P->run_len[op] = run_len;
  P->conc[op] = conc;
  return rebuild_op(P, op);
}

fc_status fc_plan_get_tuning(const fc_plan* P, int32_t op, int32_t* run_len, int32_t* conc) {
  if (!P || op < 0 || op > 4) return FC_E_ARG;
  if (run_len) *run_len = P->run_len[op];
  if (conc) *conc = P->conc[op];
  return FC_OK;
}

fc_status fc_plan_set_transform_plan(fc_plan* P, int32_t op, int32_t tplan) {
  if (!P || op < 0 || op > 4 || tplan < 0 || tplan > 1) return FC_E_ARG;
  if (!P->op[op].valid) return FC_E_STATE;
  if (P->device >= 0) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
    const bool ok = hipDeviceSynchronize() == hipSuccess;
    P->tplan[op] = tplan;
    P->class_tp[op].clear();
    const fc_status st = ok ? rebuild_op(P, op) : FC_E_DEVICE;
    (void)hipSetDevice(cur);
    return st;
  }
  P->tplan[op] = tplan;
  P->class_tp[op].clear();
  return rebuild_op(P, op);
}

fc_status fc_plan_get_class_plans(const fc_plan* P, int32_t op, int32_t* n_classes, int32_t* n_plan1) {
  if (!P || op < 0 || op > 4 || !n_classes || !n_plan1) return FC_E_ARG;
  if (!P->op[op].valid) return FC_E_STATE;
  *n_classes = 0;
  *n_plan1 = 0;
  for (const auto& ph : P->op[op].phases) {
    if (ph.kind == 2) continue;
    const bool alt = (ph.cls == 0 && pruned_has_alt(ph.size)) || ((ph.cls == 2 || ph.cls == 4) && rx_has_alt(ph.size));
    if (!alt) continue;
    ++*n_classes;
    if (ph.tplan == 1) ++*n_plan1;
  }
  return FC_OK;
}

fc_status fc_plan_get_transform_plan(const fc_plan* P, int32_t op, int32_t* tplan) {
  if (!P || op < 0 || op > 4 || !tplan) return FC_E_ARG;
  *tplan = P->tplan[op];
  return FC_OK;
}

// Whether transform plan 1 differs from plan 0 for some launch of op: a
// pruned TX class with L <= 1024, or an RX-family launch with a long FFT
// whose radix cap can be lowered.
static bool has_second_plan(const fc_plan* P, int op) {
  for (const auto& ph : P->op[op].phases) {
    if (ph.kind == 2) continue;
    if (ph.cls == 0 && pruned_has_alt(ph.size)) return true;
    if ((ph.cls == 2 || ph.cls == 4) && rx_has_alt(ph.size)) return true;
  }
  return false;
}

// Time of one call of op under the current tuning: calls back to back, as a
// caller streaming work issues them (one warm-up call, then three bursts of
// four calls between two events; the shortest burst's time per call). On a
// capturable stream the call is recorded once as a HIP graph and the graph
// is replayed, so host launch gaps between the op's kernels stay out of the
// time (they vary between runs by more than the work splits differ); on the
// legacy null stream the calls run eagerly.
static fc_status time_op(fc_plan* P, int op, const void* in, void* out, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1, float* t_min) {
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  fc_status r = FC_OK;
  if (st) {
    if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) return FC_E_DEVICE;
    r = run_op(P, op, in, out, st);
    const bool ended = hipStreamEndCapture(st, &g) == hipSuccess && g;
    if (r == FC_OK && !ended) r = FC_E_DEVICE;
    if (r == FC_OK && hipGraphInstantiate(&ge, g, nullptr, nullptr, 0) != hipSuccess) r = FC_E_DEVICE;
  }
  auto call = [&]() { return ge ? (hipGraphLaunch(ge, st) == hipSuccess ? FC_OK : FC_E_DEVICE)
                                 : run_op(P, op, in, out, st); };
  constexpr int kBurst = 4;
  *t_min = 1e30f;
  if (r == FC_OK) r = call();                               // warm-up
  for (int rep = 0; rep < 3 && r == FC_OK; ++rep) {
    if (hipEventRecord(e0, st) != hipSuccess) { r = FC_E_DEVICE; break; }
    for (int k = 0; k < kBurst && r == FC_OK; ++k) r = call();
    if (r != FC_OK) break;
    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) { r = FC_E_DEVICE; break; }
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *t_min = std::min(*t_min, ms / kBurst);
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  return r;
}

fc_status fc_plan_autotune(fc_plan* P, int32_t op, const void* in, void* out, void* stream, int32_t* best_run_len,
                           int32_t* best_conc, float* best_ms) {
  if (!P || op < 0 || op > 4 || !in || !out) return FC_E_ARG;
  if (!P->op[op].valid || P->device < 0) return FC_E_STATE;
  const hipStream_t st = (hipStream_t)stream;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  const std::vector<int> lens = (op == FC_OP_TX || op == FC_OP_TXG) ? std::vector<int>{0, 8, 16, 32, 64}
                               : op == FC_OP_RXD ? std::vector<int>{0, 2, 4, 8, 16}
                                                 : std::vector<int>{0, 1, 2, 4, 8, 16};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  fc_status result = FC_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) result = FC_E_DEVICE;
  float best = 1e30f;
  int b_len = P->run_len[op], b_conc = P->conc[op], b_tp = P->tplan[op];
  bool b_meas = false;                     // launches ordered by measured (not estimated) work
  const int n_tp = has_second_plan(P, op) ? 2 : 1;
  const auto saved_classes = P->class_tp[op];
  P->class_tp[op].clear();
  for (int tp = 0; tp < n_tp && result == FC_OK; ++tp) {
    P->tplan[op] = tp;                     // applied by the rebuilds of set_tuning below
    for (int conc : {1, kMaxConc}) {
      for (int len : lens) {
        if (result != FC_OK) break;
        if ((result = fc_plan_set_tuning(P, op, len, conc)) != FC_OK) break;
        // with several streams: the launches spread by the planner's work
        // estimate, then by each launch's measured time (neither order wins
        // on every workload)
        for (int meas = 0; meas < (conc > 1 ? 2 : 1) && result == FC_OK; ++meas) {
          if (meas && (result = measure_costs(P, op, in, out, st, e0, e1)) != FC_OK) break;
          float t_min = 1e30f;
          result = time_op(P, op, in, out, st, e0, e1, &t_min);
          if (result == FC_OK && t_min < best) {
            best = t_min; b_len = len; b_conc = conc; b_tp = tp; b_meas = meas != 0;
          }
        }
      }
    }
  }
  P->tplan[op] = b_tp;
  if (result != FC_OK) P->class_tp[op] = saved_classes;
  if (result == FC_OK) result = fc_plan_set_tuning(P, op, b_len, b_conc);
  if (result == FC_OK && b_meas) result = measure_costs(P, op, in, out, st, e0, e1);
  // then, class by class (largest first), the other transform plan where it
  // makes the whole call at least 1.5 % faster (well above the timing noise
  // of the minimum of six replays): the classes share the GPU, so each
  // change is judged on the call, not on the class
  if (result == FC_OK && n_tp == 2) {
    std::vector<std::tuple<int, int, int>> keys;
    for (const auto& ph : P->op[op].phases) {
      if (ph.kind == 2) continue;
      const bool alt = (ph.cls == 0 && pruned_has_alt(ph.size)) || ((ph.cls == 2 || ph.cls == 4) && rx_has_alt(ph.size));
      const auto key = std::make_tuple(ph.cls, ph.size, ph.key3);
      if (alt && std::find(keys.begin(), keys.end(), key) == keys.end()) keys.push_back(key);
    }
    float cur = 1e30f;
    result = time_op(P, op, in, out, st, e0, e1, &cur);
    for (size_t i = 0; i < keys.size() && result == FC_OK; ++i) {
      P->class_tp[op][keys[i]] = 1 - b_tp;
      if ((result = fc_plan_set_tuning(P, op, b_len, b_conc)) != FC_OK) break;
      if (b_meas && (result = measure_costs(P, op, in, out, st, e0, e1)) != FC_OK) break;
      float t = 1e30f;
      if ((result = time_op(P, op, in, out, st, e0, e1, &t)) != FC_OK) break;
      if (t < 0.985f * cur) cur = t;
      else P->class_tp[op].erase(keys[i]);
    }
    if (result == FC_OK) result = fc_plan_set_tuning(P, op, b_len, b_conc);
    if (result == FC_OK && b_meas) result = measure_costs(P, op, in, out, st, e0, e1);
    if (result == FC_OK) best = cur;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipSetDevice(cur);
  if (result != FC_OK) return result;
  if (best_run_len) *best_run_len = b_len;
  if (best_conc) *best_conc = b_conc;
  if (best_ms) *best_ms = best;
  return FC_OK;
}

fc_status fc_plan_stats(const fc_plan* P, int32_t op, int64_t* n_blocks, int64_t* n_tasks, int64_t* n_launches) {
  if (!P || op < FC_OP_TX || op > FC_OP_TXG) return FC_E_ARG;
  const Op& o = P->op[op];
  if (!o.valid) return FC_E_STATE;
  if (n_blocks) *n_blocks = (int64_t)o.blk.size();
  if (n_tasks) *n_tasks = (int64_t)o.task.size();
  if (n_launches) *n_launches = (int64_t)o.phases.size();
  return FC_OK;
}

fc_status fc_tx_synthesize(fc_plan* P, const void* in, void* out, void* stream) {
  if (!P) return FC_E_ARG;
  return run_op(P, FC_OP_TX, in, out, (hipStream_t)stream);
}

fc_status fc_rx_analyze(fc_plan* P, const void* in, void* out, void* stream) {
  if (!P) return FC_E_ARG;
  return run_op(P, FC_OP_RX, in, out, (hipStream_t)stream);
}

fc_status fc_tx_modulate(fc_plan* P, const void* grid_in, void* out, void* stream) {
  if (!P) return FC_E_ARG;
  return run_op(P, FC_OP_TXG, grid_in, out, (hipStream_t)stream);
}

fc_status fc_rx_demodulate(fc_plan* P, const void* in, void* out, void* stream) {
  if (!P) return FC_E_ARG;
  return run_op(P, FC_OP_RXD, in, out, (hipStream_t)stream);
}

fc_status fc_tx_adjoint(fc_plan* P, const void* in, void* out, void* stream) {
  if (!P) return FC_E_ARG;
  return run_op(P, FC_OP_ADJ, in, out, (hipStream_t)stream);
}

fc_status fc_tx_weight_grad(fc_plan* P, const void* lowrate_in, const void* grad_out, float* grad_w,
                            void* stream) {
  if (!P) return FC_E_ARG;
  return run_wgrad(P, lowrate_in, grad_out, grad_w, (hipStream_t)stream);
}

fc_status fc_tx_weight_grad_noalloc(fc_plan* P, const void* lowrate_in, const void* grad_out, float* grad_w,
                                    void* stream) {
  if (!P) return FC_E_ARG;
  const Op& op = P->op[kOpWgrad];
  if (!op.valid || P->device < 0) return FC_E_STATE;
  if (!lowrate_in || !grad_out || !grad_w) return FC_E_ARG;
  if (op.part_total > (int64_t)(FC_NOALLOC_SCRATCH_BYTES / sizeof(float))) return FC_E_LIMIT;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FC_E_DEVICE;
  if (cur != P->device && hipSetDevice(P->device) != hipSuccess) return FC_E_DEVICE;
  float* part = nullptr;
  fc_status r = noalloc_scratch(P->device, &part) == hipSuccess ? FC_OK : FC_E_DEVICE;
  if (r == FC_OK) r = launch_wgrad(P, lowrate_in, grad_out, grad_w, part, (hipStream_t)stream);
  if (cur != P->device) (void)hipSetDevice(cur);
  return r;
}

}  // extern "C"

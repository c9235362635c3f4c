// C ABI of the CGL exponential stepper: plans, operator setup, pass
// sequencing of the Tucker operator inside Strang and Lawson4 steps, and
// graph-captured runs with flag checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <new>
#include <thread>
#include <atomic>
#include <tuple>
#include <vector>

#include "../../include/cgl.h"
#include "autotune.hpp"
#include "host_numerics.hpp"
#include "kernels.hpp"
#include "plan_internal.hpp"
#include "split_layout.hpp"

using namespace cgl;

namespace {

int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

// One exponential on the device: the FP64 embedding (slot 0), or the bf16
// term planes in the layout of every split tile shape (slot = tile index).
struct DeviceOp {
  void* ptr[SPLIT_NTILES] = {};
  int Pp[SPLIT_NTILES] = {}, Kp[SPLIT_NTILES] = {};
};

struct GraphKey {
  int method;
  void* u;
  int64_t k;
  bool operator<(const GraphKey& o) const {
    return std::tie(method, u, k) < std::tie(o.method, o.u, o.k);
  }
};

}  // namespace

struct cgl_plan_s {
  int d = 0;
  int64_t n[3] = {1, 1, 1};
  int64_t N = 0;
  cgl_coeffs c{};
  double tau = 0.0;
  int precision = CGL_FP64;
  unsigned flags = 0;
  hipStream_t ustream = nullptr;  // caller's stream
  hipStream_t gstream = nullptr;  // plan-owned stream used for graph capture/replay
  hipStream_t bstream = nullptr;  // plan-owned stream of the second Lawson4 branch
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr;
  bool have_ops[3] = {false, false, false};
  CMat E[3], H[3];
  DeviceOp dE[3], dH[3];
  // split tile shape per direction and prologue kind (autotuned; batched
  // plans use tile[mu][PRO_NONE] for every pass)
  int tile[3][3] = {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}};
  // split form: Lawson4 rounds as paired passes on one stream instead of
  // two concurrent actions
  bool paired = false;
  // tile shape of the paired pass per direction (2: 64 rows, 3: 128 rows;
  // autotuned; -1 not yet chosen)
  int pair_tile[3] = {-1, -1, -1};
  // the auxiliary input of the passes being enqueued is complex128 (the
  // split4 combination of a master-state plan)
  bool aux_f64 = false;
  // intermediates of the action being enqueued in caller-provided memory
  // instead of stage[0] / stage[1] (the allocation-free Tucker variant)
  void* tmp_override[2] = {nullptr, nullptr};
  // periodic directions (Section 3.2): fft[mu] runs the Fourier pass with the
  // diagonal of exp(tau A_mu) / exp(tau A_mu / 2) (host FP64 copies fac[mu][0/1],
  // device copies in the pass precision dfac, twiddles dtw)
  bool fft[3] = {false, false, false};
  std::vector<double> fac[3][2];
  void* dfac[3][2] = {};
  void* dtw[3] = {};
  // [0], [1]: ping-pong intermediates; [2..4]: Lawson4 stage tensors; [5], [6]:
  // ping-pong intermediates of the second branch
  void* stage[7] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  unsigned* dflag = nullptr;
  unsigned* hflag = nullptr;  // pinned
  std::map<GraphKey, hipGraphExec_t> graphs;
  NlParams nl{};
  // batched plans (batch > 0): independent instances, instance j has grid
  // bn[j*d .. j*d+d-1], coefficients bnl[j], and lives at complex offset boff[j]
  // split contraction of small single-action passes (set by
  // enable_split_contraction): one workspace per concurrent branch
  bool ksplit = false;
  float* ksws[2] = {nullptr, nullptr};
  int64_t ksws_floats = 0;
  int batch = 0;
  std::vector<int64_t> bn, boff;
  std::vector<NlParams> bnl;
  std::vector<CMat> bE, bH;         // [batch*d] FP64 exponentials
  std::vector<DeviceOp> bdE, bdH;   // [batch*d]
  std::vector<char> bhave;          // [batch*d]
  BatchInstance* dinst[3] = {nullptr, nullptr, nullptr};
  BatchTile* dtiles[3][SPLIT_NTILES] = {};
  int ntiles[3][SPLIT_NTILES] = {};
  bool tables = false;
  int nwg = 0;  // persistent grid size
};

namespace {

bool ready(const cgl_plan_s* p) {
  if (p->batch > 0) {
    for (char h : p->bhave)
      if (!h) return false;
    return true;
  }
  for (int mu = 0; mu < p->d; ++mu)
    if (!p->have_ops[mu]) return false;
  return true;
}

size_t stage_bytes(const cgl_plan_s* p) {
  return static_cast<size_t>(p->N) * (p->precision == CGL_FP64 ? 16 : 8);
}

bool master(const cgl_plan_s* p) {
  return p->precision == CGL_SPLIT_BF16 && (p->flags & CGL_FLAG_FP64_MASTER);
}

size_t user_bytes(const cgl_plan_s* p) {
  return static_cast<size_t>(p->N) * ((p->precision == CGL_FP64 || master(p)) ? 16 : 8);
}

void free_op(DeviceOp& o) {
  for (auto& q : o.ptr) {
    if (q) (void)hipFree(q);
    q = nullptr;
  }
}

int upload_bytes(cgl_plan_s* p, const void* h, size_t bytes, void** dst) {
  if (hipMalloc(dst, bytes) != hipSuccess) return CGL_ENOMEM;
  if (hipMemcpyAsync(*dst, h, bytes, hipMemcpyHostToDevice, p->ustream) != hipSuccess)
    return CGL_EDEVICE;
  if (hipStreamSynchronize(p->ustream) != hipSuccess) return CGL_EDEVICE;
  return CGL_OK;
}

static_assert(SPLIT_NTILES_BATCHED <= SPLIT_MAX_TILES, "batched instance tables hold the batched tile shapes");

// Upload one exponential in the plan's device form.
int upload_op(cgl_plan_s* p, const CMat& M, DeviceOp& dst) {
  const int64_t n = M.n;
  free_op(dst);
  if (p->precision == CGL_FP64) {
    const int Pp = static_cast<int>(round_up(2 * n, F64_PT));
    const int Kp = static_cast<int>(round_up(2 * n, F64_KC));
    std::vector<double> h(static_cast<size_t>(Pp) * Kp, 0.0);
    // embedding [[Re, -Im], [Im, Re]] with columns k' = 2k + c and rows
    // permuted within 16-row blocks so that the FP64 MFMA accumulator of one
    // lane (rows g, g+4, g+8, g+12 of a block) holds (re, im) of two complex
    // outputs: block b, lane group g, register r <-> m = 8b + g + 4(r/2),
    // part r%2.  Stored with k' as the row index and p' fastest.
    auto prow = [](int64_t m, int c) {
      const int64_t ml = m % 8;
      return 16 * (m / 8) + (ml % 4) + 4 * (2 * (ml / 4) + c);
    };
    for (int64_t k = 0; k < n; ++k)
      for (int64_t m = 0; m < n; ++m) {
        const double re = M.re[m + n * k], im = M.im[m + n * k];
        h[(2 * k) * Pp + prow(m, 0)] = re;
        h[(2 * k) * Pp + prow(m, 1)] = im;
        h[(2 * k + 1) * Pp + prow(m, 0)] = -im;
        h[(2 * k + 1) * Pp + prow(m, 1)] = re;
      }
    dst.Pp[0] = Pp;
    dst.Kp[0] = Kp;
    return upload_bytes(p, h.data(), h.size() * sizeof(double), &dst.ptr[0]);
  }
  const int ntile = p->batch > 0 ? SPLIT_NTILES_BATCHED : SPLIT_NTILES;
  for (int t = 0; t < ntile; ++t) {
    std::vector<uint16_t> h;
    build_split_operator(M, SPLIT_TILES[t], h, dst.Pp[t], dst.Kp[t]);
    const int st = upload_bytes(p, h.data(), h.size() * sizeof(uint16_t), &dst.ptr[t]);
    if (st != CGL_OK) return st;
  }
  return CGL_OK;
}

// rotated: the input's contraction axis is its fastest one and the output is
// written with that axis moved to the slowest position (split form only).
int pass_batched(cgl_plan_s* p, int mu, int which, const void* in0, const void* aux, void* out0,
                 void* out1, int pro, int epi, bool in_f64, bool out_f64, hipStream_t s);

int pass(cgl_plan_s* p, int mu, int which, const void* in0, const void* aux, void* out0,
         void* out1, int pro, int epi, bool in_f64, bool out_f64, bool rotated, hipStream_t s) {
  if (p->batch > 0)
    return pass_batched(p, mu, which, in0, aux, out0, out1, pro, epi, in_f64, out_f64, s);
  const DeviceOp& op = (which == CGL_E) ? p->dE[mu] : p->dH[mu];
  int64_t R = 1;
  for (int nu = 0; nu < mu; ++nu) R *= p->n[nu];
  const int n = static_cast<int>(p->n[mu]);
  if (rotated && p->precision != CGL_SPLIT_BF16) return CGL_EINVAL;
  hipError_t e;
  if (p->fft[mu]) {
    PassFFT f{};
    f.in0 = in0;
    f.aux = aux;
    f.out0 = out0;
    f.out1 = out1;
    f.fac = p->dfac[mu][which == CGL_E ? 0 : 1];
    f.tw = static_cast<const double*>(p->dtw[mu]);
    f.R = rotated ? 1 : R;
    f.R_out = rotated ? p->N / n : R;
    f.F = p->N / n;
    f.n = n;
    f.pro = pro;
    f.epi = epi;
    // complex128 tensors: every tensor of an FP64 plan, the master state's
    // ends of a complex64 plan
    f.fp64 = p->precision == CGL_FP64 ? 1 : 0;
    f.in_f64 = (f.fp64 || in_f64) ? 1 : 0;
    f.out_f64 = (f.fp64 || out_f64) ? 1 : 0;
    f.aux_f64 = (f.fp64 || p->aux_f64) ? 1 : 0;
    f.nl = p->nl;
    f.flag = p->dflag;
    e = launch_pass_fft(f, s);
    return e == hipSuccess ? CGL_OK : CGL_EDEVICE;
  }
  if (p->precision == CGL_FP64) {
    PassF64 a{};
    a.in0 = static_cast<const double*>(in0);
    a.aux = static_cast<const double*>(aux);
    a.out0 = static_cast<double*>(out0);
    a.out1 = static_cast<double*>(out1);
    a.op = static_cast<const double*>(op.ptr[0]);
    a.R = R;
    a.F = p->N / n;
    a.n = n;
    a.Pp = op.Pp[0];
    a.Kp = op.Kp[0];
    a.pro = pro;
    a.epi = epi;
    a.nl = p->nl;
    a.flag = p->dflag;
    e = launch_pass_f64(a, s);
  } else {
    PassSplit a{};
    a.in0 = in0;
    a.aux = aux;
    a.out0 = out0;
    a.out1 = out1;
    int t = p->tile[mu][pro] >= 0 ? p->tile[mu][pro] : p->tile[mu][PRO_NONE];
    if (t < 0) t = 0;
    if (!rotated && SPLIT_TILES[t].dma) t = 1;  // the direct-to-LDS shapes need a contiguous axis
    a.op = static_cast<const uint16_t*>(op.ptr[t]);
    a.tile = t;
    a.R = rotated ? 1 : R;
    a.R_out = rotated ? p->N / n : R;
    a.F = p->N / n;
    a.n = n;
    a.Pp = op.Pp[t];
    a.Kp = op.Kp[t];
    a.pro = pro;
    a.epi = epi;
    a.in_f64 = in_f64 ? 1 : 0;
    a.out_f64 = out_f64 ? 1 : 0;
    a.aux_f64 = p->aux_f64 ? 1 : 0;
    a.nl = p->nl;
    a.flag = p->dflag;
    if (p->ksplit && SPLIT_TILES[t].dma) {
      // too few tiles to fill the chip: split the contraction so that about
      // 256 workgroups run, each over at least 4 stages
      const int PT = SPLIT_TILES[t].PT;
      const int64_t G = ((a.F + SP_FT - 1) / SP_FT) * (a.Pp / PT);
      const int nKS = a.Kp / SPLIT_TILES[t].KS;
      int S = static_cast<int>(std::min<int64_t>({4, (256 + G - 1) / G, nKS / 4}));
      if (S >= 2) {
        const int chunk = (nKS + S - 1) / S;
        S = (nKS + chunk - 1) / chunk;
        if (S >= 2 && S * G * (PT / 64) * 8192 <= p->ksws_floats) {
          a.ksplit = S;
          a.kchunk = chunk;
          a.ws = p->ksws[s == p->bstream ? 1 : 0];
          a.ws_floats = p->ksws_floats;
        }
      }
    }
    e = launch_pass_split(a, s);
  }
  return e == hipSuccess ? CGL_OK : CGL_EDEVICE;
}

// One pass over every instance of a batched plan.  Split form: one persistent
// launch over the tile table of direction mu (rotated layout).  FP64 form: one
// in-place launch per instance.
int pass_batched(cgl_plan_s* p, int mu, int which, const void* in0, const void* aux, void* out0,
                 void* out1, int pro, int epi, bool in_f64, bool out_f64, hipStream_t s) {
  const int d = p->d;
  if (p->precision == CGL_SPLIT_BF16) {
    if (!p->tables) return CGL_ENOTREADY;
    const int t = p->tile[mu][PRO_NONE] >= 0 ? p->tile[mu][PRO_NONE] : 0;
    PassBatch b{};
    b.in0 = in0;
    b.aux = aux;
    b.out0 = out0;
    b.out1 = out1;
    b.inst = p->dinst[mu];
    b.tiles = p->dtiles[mu][t];
    b.ntiles = p->ntiles[mu][t];
    b.which = which == CGL_E ? 0 : 1;
    b.pro = pro;
    b.epi = epi;
    b.in_f64 = in_f64 ? 1 : 0;
    b.out_f64 = out_f64 ? 1 : 0;
    b.aux_f64 = p->aux_f64 ? 1 : 0;
    b.tile = t;
    b.tf = p->nl.tf;
    b.flag = p->dflag;
    return launch_pass_split_batched(b, p->nwg, s) == hipSuccess ? CGL_OK : CGL_EDEVICE;
  }
  for (int j = 0; j < p->batch; ++j) {
    const int64_t* nj = &p->bn[static_cast<size_t>(j) * d];
    int64_t Nj = 1, R = 1;
    for (int nu = 0; nu < d; ++nu) Nj *= nj[nu];
    for (int nu = 0; nu < mu; ++nu) R *= nj[nu];
    const DeviceOp& op = (which == CGL_E) ? p->bdE[static_cast<size_t>(j) * d + mu]
                                          : p->bdH[static_cast<size_t>(j) * d + mu];
    const size_t o = static_cast<size_t>(p->boff[j]) * 2;
    PassF64 a{};
    a.in0 = static_cast<const double*>(in0) + o;
    a.aux = aux ? static_cast<const double*>(aux) + o : nullptr;
    a.out0 = static_cast<double*>(out0) + o;
    a.out1 = out1 ? static_cast<double*>(out1) + o : nullptr;
    a.op = static_cast<const double*>(op.ptr[0]);
    a.R = R;
    a.F = Nj / nj[mu];
    a.n = static_cast<int>(nj[mu]);
    a.Pp = op.Pp[0];
    a.Kp = op.Kp[0];
    a.pro = pro;
    a.epi = epi;
    a.nl = p->bnl[j];
    a.nl.tf = p->nl.tf;
    a.flag = p->dflag;
    if (launch_pass_f64(a, s) != hipSuccess) return CGL_EDEVICE;
  }
  return CGL_OK;
}

// Device instance tables and tile lists of a split batched plan (built once
// all operators are set).  Tiles are ordered by decreasing contraction length
// so that the persistent grid's round-robin deal balances the work.
int build_tables(cgl_plan_s* p) {
  if (p->tables || p->batch == 0 || p->precision != CGL_SPLIT_BF16) return CGL_OK;
  const int d = p->d;
  for (int mu = 0; mu < d; ++mu) {
    std::vector<BatchInstance> inst(p->batch);
    for (int j = 0; j < p->batch; ++j) {
      const size_t k = static_cast<size_t>(j) * d + mu;
      int64_t Nj = 1;
      for (int nu = 0; nu < d; ++nu) Nj *= p->bn[static_cast<size_t>(j) * d + nu];
      BatchInstance& b = inst[j];
      b.off = p->boff[j];
      b.n = static_cast<int>(p->bn[k]);
      b.F = static_cast<int>(Nj / p->bn[k]);
      for (int t = 0; t < SPLIT_NTILES_BATCHED; ++t) {
        b.Pp[t] = p->bdE[k].Pp[t];
        b.Kp[t] = p->bdE[k].Kp[t];
        b.opE[t] = static_cast<const uint16_t*>(p->bdE[k].ptr[t]);
        b.opH[t] = static_cast<const uint16_t*>(p->bdH[k].ptr[t]);
      }
      b.nl = p->bnl[j];
    }
    int st = upload_bytes(p, inst.data(), inst.size() * sizeof(BatchInstance),
                          reinterpret_cast<void**>(&p->dinst[mu]));
    if (st != CGL_OK) return st;
    for (int t = 0; t < SPLIT_NTILES_BATCHED; ++t) {
      // Groups of work items that read the same operator rows or the same
      // state tiles (all items of one instance), largest contraction first,
      // each put in the shortest of XCDS columns; the table interleaves the
      // columns (entry XCDS * r + x = item r of column x).  Workgroup w runs
      // on XCD w % XCDS and takes entries w, w + G, ..., so the items of a
      // group run at about the same time on one XCD and share its L2.
      constexpr int XCDS = 8;
      std::vector<std::pair<int, std::vector<BatchTile>>> groups;
      for (int j = 0; j < p->batch; ++j) {
        const int nP = inst[j].Pp[t] / SPLIT_TILES[t].PT;
        const int nF = (inst[j].F + SP_FT - 1) / SP_FT;
        std::vector<BatchTile> g;
        for (int ft = 0; ft < nF; ++ft)
          for (int pt = 0; pt < nP; ++pt) g.push_back(BatchTile{j, pt, ft});
        groups.push_back({inst[j].Kp[t], std::move(g)});
      }
      std::stable_sort(groups.begin(), groups.end(),
                       [](const auto& x, const auto& y) { return x.first > y.first; });
      std::vector<std::vector<BatchTile>> col(XCDS);
      for (auto& g : groups) {
        size_t x = 0;
        for (size_t c = 1; c < col.size(); ++c)
          if (col[c].size() < col[x].size()) x = c;
        for (auto& it : g.second) col[x].push_back(it);
      }
      size_t rows = 0;
      for (auto& c : col) rows = std::max(rows, c.size());
      std::vector<BatchTile> tl;
      for (size_t r = 0; r < rows; ++r)
        for (int x = 0; x < XCDS; ++x)
          tl.push_back(r < col[x].size() ? col[x][r] : BatchTile{-1, 0, 0});  // -1: no work
      p->ntiles[mu][t] = static_cast<int>(tl.size());
      st = upload_bytes(p, tl.data(), tl.size() * sizeof(BatchTile),
                        reinterpret_cast<void**>(&p->dtiles[mu][t]));
      if (st != CGL_OK) return st;
    }
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  p->nwg = 2 * cus;  // two 256-thread workgroups per CU fit the LDS of either tile shape
  p->tables = true;
  return CGL_OK;
}

// Where an exponential action stands between passes: the tensor the next
// pass reads and whether it is complex128.
struct ActionCursor {
  const void* cur;
  bool f64;
};

// Passes [mu0, mu1) of one exponential action.  Intermediate results
// alternate between the ping-pong buffers of branch br (stage[0] / stage[1],
// or stage[5] / stage[6]); the first pass applies the prologue, the last pass
// (mu = d - 1) the epilogue and writes out0 (and out1).  A pass never reads
// and writes the same buffer: with d = 1 and out0 == in0 the result goes
// through a ping-pong buffer.
int action_range(cgl_plan_s* p, int which, ActionCursor& c, const void* aux, void* out0,
                 void* out1, int pro, int epi, bool out_f64, hipStream_t s, int br, int mu0,
                 int mu1) {
  // the split form rotates the axis order by one per pass (back to the
  // original after d passes); the FP64 form contracts in place
  const bool rotated = p->precision == CGL_SPLIT_BF16;
  void* const* tmp = br == 0 ? (p->tmp_override[0] ? p->tmp_override : &p->stage[0]) : &p->stage[5];
  for (int mu = mu0; mu < mu1; ++mu) {
    const bool last = (mu == p->d - 1);
    void* dst = last ? out0 : tmp[mu & 1];
    const bool via_tmp = last && dst == c.cur;
    if (via_tmp) dst = tmp[0];
    const bool of64 = last ? out_f64 : false;
    int st = pass(p, mu, which, c.cur, aux, dst, out1, mu == 0 ? pro : PRO_NONE,
                  last ? epi : EPI_NONE, c.f64, of64, rotated, s);
    if (st != CGL_OK) return st;
    if (via_tmp) {
      // stage buffers are sized for the caller's element type (see cgl_plan)
      const size_t bytes = of64 ? static_cast<size_t>(p->N) * 16 : stage_bytes(p);
      if (hipMemcpyAsync(out0, dst, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return CGL_EDEVICE;
    }
    c.cur = dst;
    c.f64 = of64;
  }
  return CGL_OK;
}

// All d passes of one exponential action on stream s (branch 0 buffers).
int action(cgl_plan_s* p, int which, const void* in0, const void* aux, void* out0, void* out1,
           int pro, int epi, bool in_f64, bool out_f64, hipStream_t s) {
  ActionCursor c{in0, in_f64};
  return action_range(p, which, c, aux, out0, out1, pro, epi, out_f64, s, 0, 0, p->d);
}

int pass_pair(cgl_plan_s* p, int mu, int which, const void* in0, const void* in1, void* out0,
              void* out1, bool sameg, int epi, bool in_f64, bool out_f64, hipStream_t s);

// Picks the paired pass's tile shape (64 or 128 rows) of every direction by
// timing it on the plan's stream (stage buffers as scratch).  For a batched
// plan the choice covers every instance of a direction.
int tune_pair(cgl_plan_s* p) {
  const char* forced = std::getenv("CGL_PAIR_TILE");
  for (int mu = 0; mu < p->d; ++mu) {
    if (p->pair_tile[mu] >= 0) continue;
    if (forced) {
      const int t = std::atoi(forced);
      if (t != 2 && t != 3) return CGL_EINVAL;
      p->pair_tile[mu] = t;
      continue;
    }
    std::string key;
    if (p->batch > 0) {
      uint64_t h = 1469598103934665603ull;  // FNV-1a over the instance sizes
      for (int64_t v : p->bn) h = (h ^ static_cast<uint64_t>(v)) * 1099511628211ull;
      key = device_tag() + ":pairbatch:b" + std::to_string(p->batch) + ":mu" + std::to_string(mu) +
            ":h" + std::to_string(h);
    } else {
      const int64_t n = p->n[mu];
      key = device_tag() + ":pair:n" + std::to_string(n) + ":F" + std::to_string(p->N / n);
    }
    auto launch = [&](int c) -> hipError_t {
      p->pair_tile[mu] = 2 + c;
      const int st = pass_pair(p, mu, CGL_H, p->stage[0], p->stage[5], p->stage[1], p->stage[6],
                               false, EPI_NONE, false, false, p->ustream);
      p->pair_tile[mu] = -1;
      return st == CGL_OK ? hipSuccess : hipErrorInvalidValue;
    };
    p->pair_tile[mu] = 2 + autotune_pick(key, 2, launch, p->ustream, 8);
  }
  return CGL_OK;
}

// Picks the split tile shape of every direction by timing passes of each
// candidate on the plan's stream (stage buffers as scratch).  The first pass
// of an action (direction 0) carries the prologue of the stepper (the Strang
// sub-flow, or g for Lawson4), evaluated once per p-tile workgroup, so it is
// tuned separately for each prologue kind.  Runs outside any graph capture; a
// no-op for FP64 plans and choices already made.
int ensure_tuned_single(cgl_plan_s* p) {
  if (p->precision != CGL_SPLIT_BF16) return CGL_OK;
  const int bt = build_tables(p);
  if (bt != CGL_OK) return bt;
  // CGL_SPLIT_TILE=<index> fixes the tile shape (tests of every shape, tuning studies)
  const char* forced = std::getenv("CGL_SPLIT_TILE");
  const int ncand = p->batch > 0 ? SPLIT_NTILES_BATCHED : SPLIT_NTILES;
  for (int mu = 0; mu < p->d; ++mu) {
    if (p->fft[mu]) continue;  // the Fourier pass has no tile shape
    for (int pro : {PRO_NONE, PRO_FLOW, PRO_G}) {
      if (pro != PRO_NONE && (mu != 0 || p->batch > 0)) continue;
      if (p->tile[mu][pro] >= 0) continue;
      if (forced) {
        const int t = std::atoi(forced);
        if (t < 0 || t >= ncand) return CGL_EINVAL;
        p->tile[mu][pro] = t;
        continue;
      }
      std::string key;
      if (p->batch > 0) {
        uint64_t h = 1469598103934665603ull;  // FNV-1a over the instance sizes
        for (int64_t v : p->bn) h = (h ^ static_cast<uint64_t>(v)) * 1099511628211ull;
        key = device_tag() + ":splitbatch:b" + std::to_string(p->batch) + ":mu" +
              std::to_string(mu) + ":h" + std::to_string(h);
      } else {
        const int64_t n = p->n[mu];
        key = device_tag() + ":split:n" + std::to_string(n) + ":F" + std::to_string(p->N / n) +
              ":pro" + std::to_string(pro) + ":f" + std::to_string(p->nl.flow);
      }
      int saved[3];
      for (int q = 0; q < 3; ++q) saved[q] = p->tile[mu][q];
      auto launch = [&](int t) -> hipError_t {
        for (int q = 0; q < 3; ++q) p->tile[mu][q] = t;
        const int st = pass(p, mu, CGL_H, p->stage[0], nullptr, p->stage[1], nullptr, pro,
                            EPI_NONE, false, false, true, p->ustream);
        for (int q = 0; q < 3; ++q) p->tile[mu][q] = saved[q];
        return st == CGL_OK ? hipSuccess : hipErrorInvalidValue;
      };
      // Every p-tile workgroup re-reads and re-splits the state of its fibre
      // tile.  Timed alone a pass hides that cost (its input stays in
      // cache); inside a step, where two actions run side by side and every
      // pass reads what the previous one wrote, it shows: measured at 256^3,
      // 64 x 16 tiles (4 p-tiles) win a lone pass by 3% and lose the step by
      // 2-3% to 128 x 16 tiles (2 p-tiles).  Each p-tile beyond the first
      // therefore counts 4% of the measured time.
      double weight[SPLIT_NTILES];
      for (int t = 0; t < ncand; ++t) {
        const int64_t n = p->batch > 0 ? 0 : p->n[mu];
        const int64_t np = (n + SPLIT_TILES[t].PT - 1) / SPLIT_TILES[t].PT;
        weight[t] = 1.0 + 0.04 * static_cast<double>(np > 1 ? np - 1 : 0);
      }
      p->tile[mu][pro] = autotune_pick(key + ":t" + std::to_string(SPLIT_NTILES) + ":w4", ncand,
                                       launch, p->ustream, 8, weight);
    }
  }
  return CGL_OK;
}

// Strang (eq. Strang): u <- phi_{tau/2}(e^{tau K} phi_{tau/2}(u)), both sub-flows
// fused into the action (first-pass prologue, last-pass epilogue).
int enqueue_strang(cgl_plan_s* p, void* u, hipStream_t s) {
  const bool m = master(p);
  p->nl.tf = 0.5 * p->tau;
  return action(p, CGL_E, u, nullptr, u, nullptr, PRO_FLOW, EPI_FLOW, m, m, s);
}

// split4 (eq. Richardson): three actions,
//   S = phi_{tau/2}(e^{tau K} phi_{tau/2}(u))                      [the full Strang step]
//   V = mid_{tau/4}(e^{tau K/2} phi_{tau/4}(u))                    [first half step + the
//                                                                   sub-flow between halves]
//   u <- 4/3 phi_{tau/4}(e^{tau K/2} V) - 1/3 S                    [combination in the epilogue]
// S and V live in stage[2] and stage[3] (S in complex128 for a master-state
// plan, so the combination keeps FP64 inputs).
int enqueue_split4(cgl_plan_s* p, void* u, hipStream_t s) {
  const bool m = master(p);
  void* S = p->stage[2];
  void* V = p->stage[3];
  p->nl.tf = 0.5 * p->tau;
  int st = action(p, CGL_E, u, nullptr, S, nullptr, PRO_FLOW, EPI_FLOW, m, m, s);
  p->nl.tf = 0.25 * p->tau;
  if (st == CGL_OK) st = action(p, CGL_H, u, nullptr, V, nullptr, PRO_FLOW, EPI_MID, m, false, s);
  p->aux_f64 = m;
  if (st == CGL_OK) st = action(p, CGL_H, V, S, u, nullptr, PRO_NONE, EPI_RICH, false, m, s);
  p->aux_f64 = false;
  p->nl.tf = 0.5 * p->tau;
  return st;
}

// One round of two exponential actions of e^{tau K/2}: a = H in_a -> out_a,
// and b = H pro(in_b), whose epilogue reads out_a.  The first d - 1 passes of
// b do not depend on a: they run on the plan's second stream (own ping-pong
// buffers) while a runs on s; the last pass of b follows both on s.
int lawson_round(cgl_plan_s* p, int which, const void* in_a, void* out_a, bool a_in64,
                 const void* in_b, bool b_in64, int pro_b, int epi_b, void* out_b0, void* out_b1,
                 bool b_out64, hipStream_t s) {
  if (p->d == 1) {
    int st = action(p, which, in_a, nullptr, out_a, nullptr, PRO_NONE, EPI_NONE, a_in64, false, s);
    if (st == CGL_OK)
      st = action(p, which, in_b, out_a, out_b0, out_b1, pro_b, epi_b, b_in64, b_out64, s);
    return st;
  }
  if (hipEventRecord(p->ev_fork, s) != hipSuccess ||
      hipStreamWaitEvent(p->bstream, p->ev_fork, 0) != hipSuccess)
    return CGL_EDEVICE;
  ActionCursor cb{in_b, b_in64};
  int st = action_range(p, which, cb, nullptr, nullptr, nullptr, pro_b, EPI_NONE, false,
                        p->bstream, 1, 0, p->d - 1);
  const bool recorded = hipEventRecord(p->ev_join, p->bstream) == hipSuccess;
  if (st == CGL_OK)
    st = action(p, which, in_a, nullptr, out_a, nullptr, PRO_NONE, EPI_NONE, a_in64, false, s);
  // rejoin s even when an enqueue failed, so that a capture can end
  if (!recorded || hipStreamWaitEvent(s, p->ev_join, 0) != hipSuccess) return CGL_EDEVICE;
  if (st == CGL_OK)
    st = action_range(p, which, cb, out_a, out_b0, out_b1, PRO_NONE, epi_b, b_out64, s, 1,
                      p->d - 1, p->d);
  return st;
}

// One direction of both actions of a round (split form): the paired kernel
// on the 64 x 16 direct-to-LDS planes of e^{tau A_mu / 2} (which = CGL_H) or
// e^{tau A_mu} (CGL_E), for one plan or every instance of a batched plan.
int pass_pair(cgl_plan_s* p, int mu, int which, const void* in0, const void* in1, void* out0,
              void* out1, bool sameg, int epi, bool in_f64, bool out_f64, hipStream_t s) {
  const int t = p->pair_tile[mu] >= 0 ? p->pair_tile[mu] : 2;
  if (p->batch > 0) {
    if (!p->tables) return CGL_ENOTREADY;
    PassBatch b{};
    b.in0 = in0;
    b.in1 = in1;
    b.out0 = out0;
    b.out1 = out1;
    b.inst = p->dinst[mu];
    b.tiles = p->dtiles[mu][t];
    b.ntiles = p->ntiles[mu][t];
    b.which = which == CGL_E ? 0 : 1;
    b.tf = p->nl.tf;
    b.pro = sameg ? PRO_G : PRO_NONE;
    b.epi = epi;
    b.in_f64 = in_f64 ? 1 : 0;
    b.out_f64 = out_f64 ? 1 : 0;
    b.tile = t;
    b.flag = p->dflag;
    return launch_pass_split_batched_pair(b, p->nwg, s) == hipSuccess ? CGL_OK : CGL_EDEVICE;
  }
  const DeviceOp& op = which == CGL_E ? p->dE[mu] : p->dH[mu];
  const int n = static_cast<int>(p->n[mu]);
  PassSplit a{};
  a.in0 = in0;
  a.in1 = in1;
  a.out0 = out0;
  a.out1 = out1;
  a.op = static_cast<const uint16_t*>(op.ptr[t]);
  a.tile = t;
  a.R = 1;
  a.R_out = p->N / n;
  a.F = p->N / n;
  a.n = n;
  a.Pp = op.Pp[t];
  a.Kp = op.Kp[t];
  a.pro = sameg ? PRO_G : PRO_NONE;
  a.epi = epi;
  a.in_f64 = in_f64 ? 1 : 0;
  a.out_f64 = out_f64 ? 1 : 0;
  a.nl = p->nl;
  a.flag = p->dflag;
  return launch_pass_split_pair(a, s) == hipSuccess ? CGL_OK : CGL_EDEVICE;
}

// Lawson4 on one stream with paired passes: round 1 takes u to (X, Y) in d
// passes that apply e^{tau A_mu / 2} to u and g(u) together, round 2 takes
// (X, Y) to u_{n+1} in d passes; intermediate pairs alternate between
// (stage[0], stage[5]) and (stage[1], stage[6]), (X, Y) live in stage[2] and
// stage[3].
int enqueue_lawson4_paired(cgl_plan_s* p, void* u, hipStream_t s) {
  const bool m = master(p);
  const int d = p->d;
  const void* in0 = u;
  const void* in1 = u;
  for (int round = 0; round < 2; ++round) {
    for (int mu = 0; mu < d; ++mu) {
      const bool last = mu == d - 1;
      void* o0 = last ? (round == 0 ? p->stage[2] : u) : p->stage[mu & 1];
      void* o1 = last ? (round == 0 ? p->stage[3] : nullptr) : p->stage[5 + (mu & 1)];
      const int epi = last ? (round == 0 ? EPI_L4_R1 : EPI_L4_R2) : EPI_NONE;
      const int st = pass_pair(p, mu, CGL_H, in0, in1, o0, o1, round == 0 && mu == 0, epi,
                               round == 0 && mu == 0 && m, round == 1 && last && m, s);
      if (st != CGL_OK) return st;
      in0 = o0;
      in1 = o1;
    }
  }
  return CGL_OK;
}

// Lawson4 (eq. lawson4) with e^{tau K} = e^{tau K/2} e^{tau K/2}: four
// actions of e^{tau K/2} in two rounds,
//   P = H u,  Q = H g(u) -> (X, Y) in the epilogue;  H X,  H Y -> u_{n+1},
// where the stage combinations run in the last-pass epilogues.
int enqueue_lawson4(cgl_plan_s* p, void* u, hipStream_t s) {
  if (p->paired) return enqueue_lawson4_paired(p, u, s);
  const bool m = master(p);
  void* B0 = p->stage[2];
  void* B1 = p->stage[3];
  void* B2 = p->stage[4];
  int st = lawson_round(p, CGL_H, u, B0, m, u, m, PRO_G, EPI_L4_R1, B1, B2, false, s);
  if (st == CGL_OK)
    st = lawson_round(p, CGL_H, B1, B0, false, B2, false, PRO_NONE, EPI_L4_R2, u, nullptr, m, s);
  return st;
}

// Lawson2b (eq. lawson2b) with e^{tau K}(u + c g(u)) = P + c Q, P = e^{tau K} u,
// Q = e^{tau K} g(u): one round of two actions of e^{tau K}, whose last pass
// forms u_{n+1} = P + tau/2 Q + tau/2 g(P + tau Q).  Split plans run the
// round as paired passes (u and g(u) staged from one read of u); a 1-D plan's
// single pass reads u, so its result goes through stage[2].
int enqueue_lawson2(cgl_plan_s* p, void* u, hipStream_t s) {
  const bool m = master(p);
  const int d = p->d;
  if (p->paired) {
    const void* in0 = u;
    const void* in1 = u;
    for (int mu = 0; mu < d; ++mu) {
      const bool last = mu == d - 1;
      void* o0 = last ? (d == 1 ? p->stage[2] : u) : p->stage[mu & 1];
      void* o1 = last ? nullptr : p->stage[5 + (mu & 1)];
      const int st = pass_pair(p, mu, CGL_E, in0, in1, o0, o1, mu == 0, last ? EPI_L2 : EPI_NONE,
                               mu == 0 && m, last && m, s);
      if (st != CGL_OK) return st;
      in0 = o0;
      in1 = o1;
    }
    if (d == 1 && hipMemcpyAsync(u, p->stage[2], user_bytes(p), hipMemcpyDeviceToDevice, s) !=
                      hipSuccess)
      return CGL_EDEVICE;
    return CGL_OK;
  }
  return lawson_round(p, CGL_E, u, p->stage[2], m, u, m, PRO_G, EPI_L2, u, nullptr, m, s);
}

int enqueue_method(cgl_plan_s* p, int method, void* u, hipStream_t s) {
  switch (method) {
    case CGL_STRANG: return enqueue_strang(p, u, s);
    case CGL_LAWSON4: return enqueue_lawson4(p, u, s);
    case CGL_SPLIT4: return enqueue_split4(p, u, s);
    case CGL_LAWSON2: return enqueue_lawson2(p, u, s);
    default: return CGL_EINVAL;
  }
}

// Tunes what a step of `method` (or, with method < 0, a plain exponential
// action) will launch: the paired pass for the Lawson methods of a split
// plan that pairs its rounds, the single-action shapes otherwise.  Runs
// outside graph capture (it times launches).
int ensure_tuned(cgl_plan_s* p, int method) {
  if (p->precision != CGL_SPLIT_BF16) return CGL_OK;
  const bool pair = p->paired && (method == CGL_LAWSON4 || method == CGL_LAWSON2);
  if (!pair) return ensure_tuned_single(p);
  const int bt = build_tables(p);
  return bt != CGL_OK ? bt : tune_pair(p);
}

int check_u(cgl_plan_s* p, void* u, int method) {
  if (!p || !u) return CGL_EINVAL;
  if (!ready(p)) return CGL_ENOTREADY;
  if (method < CGL_STRANG || method > CGL_LAWSON2) return CGL_EINVAL;
  return ensure_tuned(p, method);
}

}  // namespace

extern "C" {

const char* cgl_strerror(int status) {
  switch (status) {
    case CGL_OK: return "ok";
    case CGL_EINVAL: return "invalid argument";
    case CGL_ENOMEM: return "out of memory";
    case CGL_EDEVICE: return "HIP runtime error";
    case CGL_ENOTREADY: return "operators not set for every direction";
    case CGL_ENONFINITE: return "state became non-finite";
    case CGL_EBLOWUP: return "exact cubic or quintic flow left its domain (blow-up)";
    case CGL_EGATE: return "surrogate jump failed its a-posteriori check";
    case CGL_ESCRATCH: return "grid too large for the allocation-free entry point's scratch";
    default: return "unknown status";
  }
}

int cgl_fd_operator(int64_t n, double a, double b, int bc, const cgl_coeffs* c, int d,
                    double* A_out) {
  if (!c || !A_out || n < 3 || d < 1 || d > 3 || !(b > a)) return CGL_EINVAL;
  if (bc != CGL_DIRICHLET && bc != CGL_NEUMANN) return CGL_EINVAL;
  const CMat A = fd_operator_2nd(n, a, b, bc, c->a1, c->b1, c->a2, d);
  A.to_interleaved(A_out);
  return CGL_OK;
}

int cgl_fd_operator_ex(int64_t n, double a, double b, int bc_lo, int bc_hi, int order,
                       const cgl_coeffs* c, int d, double* A_out) {
  if (!c || !A_out || d < 1 || d > 3 || !(b > a) || !std::isfinite(a) || !std::isfinite(b))
    return CGL_EINVAL;
  CMat A;
  if (!fd_operator(n, a, b, bc_lo, bc_hi, order, c->a1, c->b1, c->a2, d, A)) return CGL_EINVAL;
  A.to_interleaved(A_out);
  return CGL_OK;
}

int cgl_expm(int64_t n, const double* A, double t, double* out) {
  if (!A || !out || n < 1 || !std::isfinite(t)) return CGL_EINVAL;
  const CMat M = CMat::from_interleaved(n, A);
  CMat R;
  if (!expm_pade13(M, t, R)) return CGL_EINVAL;
  R.to_interleaved(out);
  return CGL_OK;
}

}  // extern "C"

namespace {

// Sub-flow of the splitting schemes: the three-term exact flows when asked
// for, the exact cubic flow (eq. exsolcub) for a cubic equation unless the
// RK4 sub-flow is forced, one RK4 step otherwise.
int flow_kind(const cgl_coeffs& c, unsigned flags) {
  if (flags & CGL_FLAG_THREE_TERM) return FLOW_3T;
  return (c.a4 == 0.0 && c.b4 == 0.0 && !(flags & CGL_FLAG_RK4_FLOW)) ? FLOW_EXACT : FLOW_RK4;
}

// Validates the common arguments and allocates a plan whose state tensors
// have N complex points (stage buffers, flags, streams, events).
int create_plan(cgl_plan_t* out, int d, const int64_t* n, int64_t N, const cgl_coeffs* c,
                double tau, int precision, unsigned flags, void* hip_stream) {
  *out = nullptr;
  if (!(tau > 0.0) || !std::isfinite(tau)) return CGL_EINVAL;
  if (!(c->a1 > 0.0)) return CGL_EINVAL;
  if (precision != CGL_FP64 && precision != CGL_SPLIT_BF16) return CGL_EINVAL;
  if (flags & ~(CGL_FLAG_FP64_MASTER | CGL_FLAG_RK4_FLOW | CGL_FLAG_THREE_TERM)) return CGL_EINVAL;
  if ((flags & CGL_FLAG_RK4_FLOW) && (flags & CGL_FLAG_THREE_TERM)) return CGL_EINVAL;
  if ((flags & CGL_FLAG_FP64_MASTER) && precision != CGL_SPLIT_BF16) return CGL_EINVAL;
  const double cv[7] = {c->a1, c->b1, c->a2, c->a3, c->b3, c->a4, c->b4};
  for (double v : cv)
    if (!std::isfinite(v)) return CGL_EINVAL;
  if (N < 3 || N > (int64_t(1) << 31)) return CGL_EINVAL;
  cgl_plan_s* p = new (std::nothrow) cgl_plan_s();
  if (!p) return CGL_ENOMEM;
  p->d = d;
  for (int mu = 0; mu < d; ++mu) p->n[mu] = n ? n[mu] : 1;
  p->N = N;
  p->c = *c;
  p->tau = tau;
  p->precision = precision;
  p->flags = flags;
  p->ustream = static_cast<hipStream_t>(hip_stream);
  p->nl.tau = tau;
  p->nl.tf = 0.5 * tau;
  p->nl.a3 = c->a3;
  p->nl.b3 = c->b3;
  p->nl.a4 = c->a4;
  p->nl.b4 = c->b4;
  p->nl.flow = flow_kind(*c, flags);
  int st = CGL_OK;
  if (hipStreamCreateWithFlags(&p->gstream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&p->bstream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess)
    st = CGL_EDEVICE;
  for (int i = 0; i < 7 && st == CGL_OK; ++i)
    if (hipMalloc(&p->stage[i], std::max(stage_bytes(p), user_bytes(p))) != hipSuccess)
      st = CGL_ENOMEM;
  if (st == CGL_OK && hipMalloc(reinterpret_cast<void**>(&p->dflag), 256) != hipSuccess)
    st = CGL_ENOMEM;
  if (st == CGL_OK && hipHostMalloc(reinterpret_cast<void**>(&p->hflag), 64) != hipSuccess)
    st = CGL_ENOMEM;
  if (st == CGL_OK && hipMemsetAsync(p->dflag, 0, 256, p->ustream) != hipSuccess)
    st = CGL_EDEVICE;
  for (int i = 0; i < 7 && st == CGL_OK; ++i)
    if (hipMemsetAsync(p->stage[i], 0, std::max(stage_bytes(p), user_bytes(p)), p->ustream) !=
        hipSuccess)
      st = CGL_EDEVICE;
  if (st == CGL_OK && hipStreamSynchronize(p->ustream) != hipSuccess) st = CGL_EDEVICE;
  if (st != CGL_OK) {
    cgl_destroy(p);
    return st;
  }
  *out = p;
  return CGL_OK;
}

}  // namespace

extern "C" {

int cgl_plan(cgl_plan_t* out, int d, const int64_t* n, const cgl_coeffs* c, double tau,
             int precision, unsigned flags, void* hip_stream) {
  if (!out) return CGL_EINVAL;
  *out = nullptr;
  if (!n || !c || d < 1 || d > 3) return CGL_EINVAL;
  int64_t N = 1;
  for (int mu = 0; mu < d; ++mu) {
    if (n[mu] < 3 || n[mu] > 4096) return CGL_EINVAL;
    N *= n[mu];
  }
  const int st = create_plan(out, d, n, N, c, tau, precision, flags, hip_stream);
  if (st == CGL_OK && precision == CGL_SPLIT_BF16) {
    // CGL_LAWSON_PAIRED=0 keeps the two concurrent actions (comparison runs)
    const char* e = std::getenv("CGL_LAWSON_PAIRED");
    (*out)->paired = !(e && e[0] == '0');
  }
  return st;
}

}  // extern "C"

namespace {

// H = exp(tau A / 2) by Pade-13 with scaling and squaring, and E = H H (the
// final squaring of the same method), for a list of operators, in parallel
// host threads.  Returns false if any exponential fails.
bool exponentials(const std::vector<CMat>& A, double tau, std::vector<CMat>& E,
                  std::vector<CMat>& H) {
  E.assign(A.size(), CMat());
  H.assign(A.size(), CMat());
  std::atomic<size_t> next{0};
  std::atomic<bool> ok{true};
  auto work = [&]() {
    for (size_t i = next++; i < A.size(); i = next++) {
      if (!expm_pade13(A[i], 0.5 * tau, H[i])) {
        ok = false;
        continue;
      }
      cmat_mul(H[i], H[i], E[i]);
    }
  };
  const unsigned hw = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 32u));
  const unsigned nt = static_cast<unsigned>(std::min<size_t>(hw, A.size()));
  std::vector<std::thread> th;
  for (unsigned t = 1; t < nt; ++t) th.emplace_back(work);
  work();
  for (auto& t : th) t.join();
  return ok;
}

bool finite_mat(const double* A, int64_t n) {
  for (int64_t k = 0; k < 2 * n * n; ++k)
    if (!std::isfinite(A[k])) return false;
  return true;
}

int set_instance(cgl_plan_s* p, size_t k, const CMat& E, const CMat& H) {
  p->bE[k] = E;
  p->bH[k] = H;
  int st = upload_op(p, E, p->bdE[k]);
  if (st == CGL_OK) st = upload_op(p, H, p->bdH[k]);
  p->bhave[k] = (st == CGL_OK);
  return st;
}

void invalidate(cgl_plan_s* p) {
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  for (int mu = 0; mu < 3; ++mu) {
    if (p->dinst[mu]) (void)hipFree(p->dinst[mu]);
    p->dinst[mu] = nullptr;
    for (int t = 0; t < SPLIT_NTILES; ++t) {
      if (p->dtiles[mu][t]) (void)hipFree(p->dtiles[mu][t]);
      p->dtiles[mu][t] = nullptr;
    }
  }
  p->tables = false;
}

}  // namespace

extern "C" {

int cgl_plan_batched(cgl_plan_t* out, int batch, int d, const int64_t* n, const cgl_coeffs* c,
                     double tau, int precision, unsigned flags, void* hip_stream) {
  if (!out) return CGL_EINVAL;
  *out = nullptr;
  if (batch < 1 || !n || !c || d < 1 || d > 3) return CGL_EINVAL;
  std::vector<int64_t> boff(batch);
  int64_t N = 0;
  for (int j = 0; j < batch; ++j) {
    int64_t Nj = 1;
    for (int mu = 0; mu < d; ++mu) {
      const int64_t v = n[static_cast<size_t>(j) * d + mu];
      if (v < 3 || v > 4096) return CGL_EINVAL;
      Nj *= v;
    }
    if (!(c[j].a1 > 0.0)) return CGL_EINVAL;
    for (double v : {c[j].a1, c[j].b1, c[j].a2, c[j].a3, c[j].b3, c[j].a4, c[j].b4})
      if (!std::isfinite(v)) return CGL_EINVAL;
    boff[j] = N;
    N += Nj;
  }
  cgl_plan_t p = nullptr;
  int st = create_plan(&p, d, nullptr, N, &c[0], tau, precision, flags, hip_stream);
  if (st != CGL_OK) return st;
  p->batch = batch;
  if (precision == CGL_SPLIT_BF16) {  // as for single plans (CGL_LAWSON_PAIRED=0: two actions)
    const char* e = std::getenv("CGL_LAWSON_PAIRED");
    p->paired = !(e && e[0] == '0');
  }
  p->bn.assign(n, n + static_cast<size_t>(batch) * d);
  p->boff = boff;
  p->bnl.resize(batch);
  for (int j = 0; j < batch; ++j) {
    NlParams q = p->nl;
    q.a3 = c[j].a3;
    q.b3 = c[j].b3;
    q.a4 = c[j].a4;
    q.b4 = c[j].b4;
    q.flow = flow_kind(c[j], flags);
    p->bnl[j] = q;
  }
  const size_t K = static_cast<size_t>(batch) * d;
  p->bE.resize(K);
  p->bH.resize(K);
  p->bdE.resize(K);
  p->bdH.resize(K);
  p->bhave.assign(K, 0);
  *out = p;
  return CGL_OK;
}

int cgl_batch_size(cgl_plan_t p, int* batch) {
  if (!p || !batch) return CGL_EINVAL;
  *batch = p->batch;
  return CGL_OK;
}

int cgl_instance_offset(cgl_plan_t p, int j, int64_t* off) {
  if (!p || !off || j < 0 || j >= std::max(1, p->batch)) return CGL_EINVAL;
  *off = p->batch > 0 ? p->boff[j] : 0;
  return CGL_OK;
}

int cgl_set_instance_operators(cgl_plan_t p, int j, int mu, const double* A) {
  if (!p || !A || p->batch == 0 || j < 0 || j >= p->batch || mu < 0 || mu >= p->d)
    return CGL_EINVAL;
  const size_t k = static_cast<size_t>(j) * p->d + mu;
  const int64_t n = p->bn[k];
  if (!finite_mat(A, n)) return CGL_EINVAL;
  std::vector<CMat> Av{CMat::from_interleaved(n, A)}, E, H;
  if (!exponentials(Av, p->tau, E, H)) return CGL_EINVAL;
  invalidate(p);
  return set_instance(p, k, E[0], H[0]);
}

int cgl_set_operators_all(cgl_plan_t p, const double* const* A) {
  if (!p || !A) return CGL_EINVAL;
  const size_t K = p->batch > 0 ? static_cast<size_t>(p->batch) * p->d : static_cast<size_t>(p->d);
  std::vector<CMat> Av(K);
  for (size_t k = 0; k < K; ++k) {
    const int64_t n = p->batch > 0 ? p->bn[k] : p->n[k];
    if (!A[k] || !finite_mat(A[k], n)) return CGL_EINVAL;
    Av[k] = CMat::from_interleaved(n, A[k]);
  }
  std::vector<CMat> E, H;
  if (!exponentials(Av, p->tau, E, H)) return CGL_EINVAL;
  invalidate(p);
  for (size_t k = 0; k < K; ++k) {
    int st;
    if (p->batch > 0) {
      st = set_instance(p, k, E[k], H[k]);
    } else {
      p->E[k] = E[k];
      p->H[k] = H[k];
      p->fft[k] = false;
      st = upload_op(p, p->E[k], p->dE[k]);
      if (st == CGL_OK) st = upload_op(p, p->H[k], p->dH[k]);
      p->have_ops[k] = (st == CGL_OK);
    }
    if (st != CGL_OK) return st;
  }
  return CGL_OK;
}

int cgl_get_instance_operator(cgl_plan_t p, int j, int mu, int which, double* out_host) {
  if (!p || !out_host || p->batch == 0 || j < 0 || j >= p->batch || mu < 0 || mu >= p->d ||
      (which != CGL_E && which != CGL_H))
    return CGL_EINVAL;
  const size_t k = static_cast<size_t>(j) * p->d + mu;
  if (!p->bhave[k]) return CGL_ENOTREADY;
  (which == CGL_E ? p->bE[k] : p->bH[k]).to_interleaved(out_host);
  return CGL_OK;
}

int cgl_set_exponentials(cgl_plan_t p, int mu, const double* E, const double* H) {
  if (!p || !E || !H || mu < 0 || mu >= p->d || p->batch > 0) return CGL_EINVAL;
  const int64_t n = p->n[mu];
  for (int64_t k = 0; k < 2 * n * n; ++k)
    if (!std::isfinite(E[k]) || !std::isfinite(H[k])) return CGL_EINVAL;
  p->E[mu] = CMat::from_interleaved(n, E);
  p->H[mu] = CMat::from_interleaved(n, H);
  p->fft[mu] = false;
  int st = upload_op(p, p->E[mu], p->dE[mu]);
  if (st == CGL_OK) st = upload_op(p, p->H[mu], p->dH[mu]);
  p->have_ops[mu] = (st == CGL_OK);
  // graphs captured before hold the old operator pointers
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  return st;
}

int cgl_set_operators(cgl_plan_t p, int mu, const double* A) {
  if (!p || !A || mu < 0 || mu >= p->d || p->batch > 0) return CGL_EINVAL;
  const int64_t n = p->n[mu];
  if (!finite_mat(A, n)) return CGL_EINVAL;
  std::vector<CMat> Av{CMat::from_interleaved(n, A)}, E, H;
  if (!exponentials(Av, p->tau, E, H)) return CGL_EINVAL;
  std::vector<double> e(2 * n * n), h(2 * n * n);
  E[0].to_interleaved(e.data());
  H[0].to_interleaved(h.data());
  return cgl_set_exponentials(p, mu, e.data(), h.data());
}

int cgl_set_periodic(cgl_plan_t p, int mu, double a, double b) {
  return set_periodic_adv(p, mu, a, b, 0.0);
}

}  // extern "C"

// cgl_set_periodic with an advection term adv d_mu in A_mu (the coupled
// system of Section 4.4 carries +-a0 d_1)
int cgl::set_periodic_adv(cgl_plan_t p, int mu, double a, double b, double adv) {
  if (!p || mu < 0 || mu >= p->d || p->batch > 0 || !(b > a) || !std::isfinite(a) ||
      !std::isfinite(b) || !std::isfinite(adv))
    return CGL_EINVAL;
  const int64_t n = p->n[mu];
  const cgl_coeffs& c = p->c;
  fourier_factors(n, a, b, c.a1, c.b1, c.a2, p->d, p->tau, p->fac[mu][0], adv);
  fourier_factors(n, a, b, c.a1, c.b1, c.a2, p->d, 0.5 * p->tau, p->fac[mu][1], adv);
  // the dense exponentials: returned by cgl_get_operator, and applied by the
  // mu-mode product kernels when n has no Fourier pass
  p->E[mu] = circulant_from_factors(n, p->fac[mu][0]);
  p->H[mu] = circulant_from_factors(n, p->fac[mu][1]);
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.second);
  p->graphs.clear();
  if (!fft_length_supported(n)) {
    p->fft[mu] = false;
    int st = upload_op(p, p->E[mu], p->dE[mu]);
    if (st == CGL_OK) st = upload_op(p, p->H[mu], p->dH[mu]);
    p->have_ops[mu] = (st == CGL_OK);
    return st;
  }
  for (int w = 0; w < 2; ++w) {
    if (p->dfac[mu][w]) (void)hipFree(p->dfac[mu][w]);
    p->dfac[mu][w] = nullptr;
    int st;
    if (p->precision == CGL_FP64) {
      st = upload_bytes(p, p->fac[mu][w].data(), p->fac[mu][w].size() * sizeof(double),
                        &p->dfac[mu][w]);
    } else {
      std::vector<float> f(p->fac[mu][w].begin(), p->fac[mu][w].end());
      st = upload_bytes(p, f.data(), f.size() * sizeof(float), &p->dfac[mu][w]);
    }
    if (st != CGL_OK) return st;
  }
  std::vector<double> tw;
  fft_twiddles(n, tw);
  if (p->dtw[mu]) (void)hipFree(p->dtw[mu]);
  p->dtw[mu] = nullptr;
  const int st = upload_bytes(p, tw.data(), tw.size() * sizeof(double), &p->dtw[mu]);
  if (st != CGL_OK) return st;
  p->fft[mu] = true;
  p->paired = false;  // the paired pass is a mu-mode product kernel: Lawson rounds as two actions
  p->have_ops[mu] = true;
  return CGL_OK;
}

extern "C" {

int cgl_get_periodic_factor(cgl_plan_t p, int mu, int which, double* out_host) {
  if (!p || !out_host || mu < 0 || mu >= p->d || (which != CGL_E && which != CGL_H) ||
      p->batch > 0)
    return CGL_EINVAL;
  const std::vector<double>& f = p->fac[mu][which == CGL_E ? 0 : 1];
  if (f.empty()) return CGL_ENOTREADY;
  std::memcpy(out_host, f.data(), f.size() * sizeof(double));
  return CGL_OK;
}

int cgl_get_operator(cgl_plan_t p, int mu, int which, double* out_host) {
  if (!p || !out_host || mu < 0 || mu >= p->d || (which != CGL_E && which != CGL_H) ||
      p->batch > 0)
    return CGL_EINVAL;
  if (!p->have_ops[mu]) return CGL_ENOTREADY;
  (which == CGL_E ? p->E[mu] : p->H[mu]).to_interleaved(out_host);
  return CGL_OK;
}

int cgl_split_terms(cgl_plan_t p, int* op_terms, int* state_terms) {
  if (!p) return CGL_EINVAL;
  if (op_terms) *op_terms = p->precision == CGL_SPLIT_BF16 ? SP_TERMS : 0;
  if (state_terms) *state_terms = p->precision == CGL_SPLIT_BF16 ? SP_TERMS : 0;
  return CGL_OK;
}

int cgl_mode_product(cgl_plan_t p, int mu, int which, const void* in_dev, void* out_dev) {
  if (!p || !in_dev || !out_dev || mu < 0 || mu >= p->d || in_dev == out_dev || p->batch > 0)
    return CGL_EINVAL;
  if (which != CGL_E && which != CGL_H) return CGL_EINVAL;
  if (!ready(p)) return CGL_ENOTREADY;
  const int st = ensure_tuned(p, -1);
  if (st != CGL_OK) return st;
  return pass(p, mu, which, in_dev, nullptr, out_dev, nullptr, PRO_NONE, EPI_NONE, false, false,
              false, p->ustream);
}

int cgl_tucker(cgl_plan_t p, int which, const void* in_dev, void* out_dev) {
  if (!p || !in_dev || !out_dev || (which != CGL_E && which != CGL_H)) return CGL_EINVAL;
  if (!ready(p)) return CGL_ENOTREADY;
  const int st = ensure_tuned(p, -1);
  if (st != CGL_OK) return st;
  return action(p, which, in_dev, nullptr, out_dev, nullptr, PRO_NONE, EPI_NONE, false, false,
                p->ustream);
}

int cgl_step_strang(cgl_plan_t p, void* u_dev, int64_t nsteps) {
  int st = check_u(p, u_dev, CGL_STRANG);
  if (st != CGL_OK) return st;
  if (nsteps < 0) return CGL_EINVAL;
  for (int64_t i = 0; i < nsteps && st == CGL_OK; ++i) st = enqueue_strang(p, u_dev, p->ustream);
  return st;
}

int cgl_step_lawson4(cgl_plan_t p, void* u_dev, int64_t nsteps) {
  int st = check_u(p, u_dev, CGL_LAWSON4);
  if (st != CGL_OK) return st;
  if (nsteps < 0) return CGL_EINVAL;
  for (int64_t i = 0; i < nsteps && st == CGL_OK; ++i) st = enqueue_lawson4(p, u_dev, p->ustream);
  return st;
}

int cgl_step(cgl_plan_t p, int method, void* u_dev, int64_t nsteps) {
  int st = check_u(p, u_dev, method);
  if (st != CGL_OK) return st;
  if (nsteps < 0) return CGL_EINVAL;
  for (int64_t i = 0; i < nsteps && st == CGL_OK; ++i)
    st = enqueue_method(p, method, u_dev, p->ustream);
  return st;
}

int cgl_clear_status(cgl_plan_t p) {
  if (!p) return CGL_EINVAL;
  return launch_clear_flag(p->dflag, p->ustream) == hipSuccess ? CGL_OK : CGL_EDEVICE;
}

static int read_flag(cgl_plan_t p, hipStream_t s, bool clear) {
  if (hipMemcpyAsync(p->hflag, p->dflag, sizeof(unsigned), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return CGL_EDEVICE;
  if (clear && launch_clear_flag(p->dflag, s) != hipSuccess) return CGL_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return CGL_EDEVICE;
  const unsigned f = *p->hflag;
  if (f & FLAG_NONFINITE) return CGL_ENONFINITE;
  if (f & FLAG_BLOWUP) return CGL_EBLOWUP;
  return CGL_OK;
}

int cgl_status(cgl_plan_t p) {
  if (!p) return CGL_EINVAL;
  return read_flag(p, p->ustream, true);
}

static int get_graph(cgl_plan_t p, int method, void* u, int64_t k, hipGraphExec_t* out) {
  const GraphKey key{method, u, k};
  auto it = p->graphs.find(key);
  if (it != p->graphs.end()) {
    *out = it->second;
    return CGL_OK;
  }
  if (hipStreamBeginCapture(p->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return CGL_EDEVICE;
  int st = CGL_OK;
  for (int64_t i = 0; i < k && st == CGL_OK; ++i) st = enqueue_method(p, method, u, p->gstream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(p->gstream, &g);
  if (st != CGL_OK || e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return st != CGL_OK ? st : CGL_EDEVICE;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return CGL_EDEVICE;
  p->graphs[key] = ex;
  *out = ex;
  return CGL_OK;
}

int cgl_run(cgl_plan_t p, int method, void* u_dev, int64_t nsteps, int64_t check_every) {
  int st = check_u(p, u_dev, method);
  if (st != CGL_OK) return st;
  if (nsteps < 0) return CGL_EINVAL;
  if (nsteps == 0) return CGL_OK;
  const int64_t k = (check_every <= 0 || check_every > nsteps) ? nsteps : check_every;
  // join the caller's stream; conditions latched before this run were
  // reported already (or are the caller's to read with cgl_status first)
  if (hipEventRecord(p->ev_in, p->ustream) != hipSuccess) return CGL_EDEVICE;
  if (hipStreamWaitEvent(p->gstream, p->ev_in, 0) != hipSuccess) return CGL_EDEVICE;
  if (launch_clear_flag(p->dflag, p->gstream) != hipSuccess) return CGL_EDEVICE;
  int64_t done = 0;
  while (done < nsteps && st == CGL_OK) {
    const int64_t chunk = std::min(k, nsteps - done);
    hipGraphExec_t ex = nullptr;
    st = get_graph(p, method, u_dev, chunk, &ex);
    if (st != CGL_OK) break;
    if (hipGraphLaunch(ex, p->gstream) != hipSuccess) {
      st = CGL_EDEVICE;
      break;
    }
    done += chunk;
    if (check_every > 0 || done == nsteps) st = read_flag(p, p->gstream, false);
  }
  if (hipEventRecord(p->ev_out, p->gstream) != hipSuccess) return CGL_EDEVICE;
  if (hipStreamWaitEvent(p->ustream, p->ev_out, 0) != hipSuccess) return CGL_EDEVICE;
  return st;
}

void cgl_destroy(cgl_plan_t p) {
  if (!p) return;
  if (p->ustream) (void)hipStreamSynchronize(p->ustream);
  if (p->gstream) (void)hipStreamSynchronize(p->gstream);
  if (p->bstream) (void)hipStreamSynchronize(p->bstream);
  (void)hipDeviceSynchronize();
  for (auto& kv : p->graphs) (void)hipGraphExecDestroy(kv.second);
  p->graphs.clear();
  for (int mu = 0; mu < 3; ++mu) {
    free_op(p->dE[mu]);
    free_op(p->dH[mu]);
    for (void* q : {p->dfac[mu][0], p->dfac[mu][1], p->dtw[mu]})
      if (q) (void)hipFree(q);
  }
  invalidate(p);
  for (auto& o : p->bdE) free_op(o);
  for (auto& o : p->bdH) free_op(o);
  for (void* s : p->stage)
    if (s) (void)hipFree(s);
  for (float* w : p->ksws)
    if (w) (void)hipFree(w);
  if (p->dflag) (void)hipFree(p->dflag);
  if (p->hflag) (void)hipHostFree(p->hflag);
  if (p->ev_in) (void)hipEventDestroy(p->ev_in);
  if (p->ev_out) (void)hipEventDestroy(p->ev_out);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->gstream) (void)hipStreamDestroy(p->gstream);
  if (p->bstream) (void)hipStreamDestroy(p->bstream);
  delete p;
}

}  // extern "C"

int cgl::enable_split_contraction(cgl_plan_t p) {
  if (!p) return CGL_EINVAL;
  if (p->precision != CGL_SPLIT_BF16 || p->batch > 0) return CGL_OK;
  const char* env = std::getenv("CGL_KSPLIT");
  if (env && std::strcmp(env, "0") == 0) return CGL_OK;
  // the largest workspace a pass can ask for: 4 splits of every tile of the
  // direct-to-LDS shapes (64 or 128 rows x 64 fibres), 8192 floats per 64 rows
  int64_t need = 0;
  for (int mu = 0; mu < p->d; ++mu) {
    const int64_t n = p->n[mu], F = p->N / n;
    need = std::max<int64_t>(need, 4 * ((n + 63) / 64 + 1) * ((F + SP_FT - 1) / SP_FT) * 8192);
  }
  for (float*& w : p->ksws)
    if (!w && hipMalloc(reinterpret_cast<void**>(&w), static_cast<size_t>(need) * sizeof(float)) !=
                  hipSuccess)
      return CGL_ENOMEM;
  p->ksws_floats = need;
  p->ksplit = true;
  return CGL_OK;
}

int cgl::tucker_with_scratch(cgl_plan_t p, int which, const void* in_dev, void* out_dev,
                             void* tmp0, void* tmp1) {
  if (!p || !in_dev || !out_dev || !tmp0 || !tmp1 || (which != CGL_E && which != CGL_H) ||
      p->batch > 0)
    return CGL_EINVAL;
  if (!ready(p)) return CGL_ENOTREADY;
  // no tuning here (it times launches): the shape chosen by an earlier call
  // of the plan, else the default shape
  p->tmp_override[0] = tmp0;
  p->tmp_override[1] = tmp1;
  const int st = action(p, which, in_dev, nullptr, out_dev, nullptr, PRO_NONE, EPI_NONE, false,
                        false, p->ustream);
  p->tmp_override[0] = p->tmp_override[1] = nullptr;
  return st;
}

int cgl::plan_info(cgl_plan_t p, PlanInfo* out) {
  if (!p || !out) return CGL_EINVAL;
  out->d = p->d;
  for (int mu = 0; mu < 3; ++mu) out->n[mu] = p->n[mu];
  out->precision = p->precision;
  out->flags = p->flags;
  out->batch = p->batch;
  out->stream = p->ustream;
  return CGL_OK;
}

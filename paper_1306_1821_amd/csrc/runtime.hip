// Host runtime of libhmc: the C-ABI of include/hmc.h.
//
// A context holds one or more chains.  Every stage of a trajectory or sweep is
// one kernel launch over the tiles of all chains (the per-chain descriptors
// live in one device array); per-chain scalar work (energy sums, Metropolis
// tests, Gibbs draws) runs in one block per chain.  Nothing in a sweep needs
// the host until its statistics are copied back at the end.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hmc.h"
#include "common.hpp"
#include "kernels.hpp"
#include "rng.hpp"

using namespace hmc;

namespace {

thread_local std::string g_err = "";

struct Chain {
  hmc_config cfg;
  hmc_buffers buf;
  bool learned = false;  // learned mass installed (hmc_set_mass)
  ChainDev dev;          // host copy of the device descriptor
  ChainDev* solo;        // device descriptor with tile bases at zero
  std::vector<double> hp;  // host mirror of the parameter block
};

struct WsLayout {
  size_t T, bdk, bgk, drn, part, shpart, mpart, T2, T3, shat, smass, lut, obs, total;
  int maxtiles;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int tiles_of(int cls, int n) {
  const long long nv = (long long)n * n * n, nh = (long long)n * n * (n / 2 + 1);
  switch (cls) {
    case kTileXY: return xpass_tiles(n);
    case kTileZ: return zpass_tiles(n);
    case kTileR: return (int)((nv + kElemPerTile - 1) / kElemPerTile);
    case kTileK: return (int)((nh + kElemPerTile - 1) / kElemPerTile);
  }
  return 0;
}

WsLayout layout(const hmc_config& c) {
  WsLayout L{};
  const int n = c.n;
  const size_t nv = (size_t)n * n * n, nh = (size_t)n * n * (n / 2 + 1);
  int mt = 0;
  for (int k = 0; k < kTileClasses; ++k) mt = std::max(mt, tiles_of(k, n));
  L.maxtiles = mt;
  size_t off = 0;
  L.T = off; off = align256(off + nh * 8);
  L.bdk = off; off = align256(off + nh * 8);
  L.bgk = off; off = align256(off + nh * 8);
  L.drn = off; off = align256(off + nv * 4);
  L.part = off; off = align256(off + (size_t)kPartSlots * mt * 8);
  L.shpart = off; off = align256(off + (size_t)mt * c.n_bins * 8);
  L.mpart = off; off = align256(off + (size_t)mt * std::max(3 * c.n_sub, c.n_bins) * 8);
  // learned mass: two more intermediate grids, F(D^(1/2)) and D^(1/2)
  L.T2 = off; off = align256(off + nh * 8);
  L.T3 = off; off = align256(off + nh * 8);
  L.shat = off; off = align256(off + nh * 8);
  L.smass = off; off = align256(off + nv * 4);
  L.lut = off; off = align256(off + 3 * (size_t)(c.n / 2) * (c.n / 2) + 1);
  L.obs = off; off = align256(off + nv / 256 * 8);  // one bit per 4 voxels
  L.total = off;
  return L;
}

bool valid_cfg(const hmc_config* c, std::string* why) {
  if (!c) { *why = "null config"; return false; }
  if (!supported_n(c->n)) { *why = "N must be one of 8, 16, 32, 64, 128, 192, 256"; return false; }
  if (c->n_sub < 1 || c->n_sub > kMaxSub) { *why = "n_sub must be in 1..32"; return false; }
  if (c->n_bins < 1 || c->n_bins > kMaxBins) { *why = "n_bins must be in 1..128"; return false; }
  if (!(c->box > 0)) { *why = "box must be positive"; return false; }
  if (c->n_leapfrog < 1) { *why = "n_leapfrog must be >= 1"; return false; }
  if (!(c->eps > 0) || !std::isfinite(c->eps)) { *why = "eps must be positive"; return false; }
  if (c->chain_id >= (1u << 24)) { *why = "chain_id must be < 2^24"; return false; }
  return true;
}

}  // namespace

struct hmc_ctx {
  std::vector<Chain> ch;
  hipStream_t stream = nullptr;
  ChainDev* d_all = nullptr;
  float2* tw = nullptr;
  double* pinned = nullptr;  // staging for host results
  int total[kTileClasses] = {0, 0, 0, 0};
  int lds_x = 0, lds_z = 0;
  int grid[3] = {0, 0, 0};  // launch grid per pass class (x, y, z); 0: one workgroup per tile
  int nsteps = 0;      // n_leapfrog (the maximum when tau_mode draws the step count)
  int cur_steps = 0;   // steps of the current trajectory / sweep
  int tau_mode = 0;
  int uniform_n = 0;  // N shared by every chain (0 if sizes differ)
  int max_nb = 0, max_sub = 0;
  // batches of several grid sizes: one descriptor array per size (tile bases from
  // zero) so that a pass class can run as one single-size launch per size group
  struct Group {
    int n = 0, nch = 0;
    int total[kTileClasses] = {0, 0, 0, 0};
    std::vector<int> members;
    ChainDev* d = nullptr;
  };
  std::vector<Group> groups;
  bool grouped[3] = {false, false, false};  // per pass class (x, y, z)
  int plan[3] = {0, 0, 0};  // radix plan per pass class for single-size launches
  bool plane_pass = true;   // fused y-z plane pass where the grid size has one
  bool learned = false;      // every chain runs the learned mass
  bool mass_mixed = false;   // some chains only have a learned mass: no trajectories
  // pass timing (hmc_timing)
  bool timing = false;
  int timing_mask = 0xf;  // pass classes that record events
  int timing_stride = 1;  // events around every timing_stride-th launch of a class
  long long timing_seen[4] = {0, 0, 0, 0};
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  double t_ms[4] = {0, 0, 0, 0};
  long long t_n[4] = {0, 0, 0, 0};
  // Philox draw index in device memory; graph replay of trajectories / sweeps
  uint32_t* d_draw = nullptr;
  bool use_graph = false;
  hipStream_t gstream = nullptr;
  hipEvent_t gev_a = nullptr, gev_b = nullptr;
  std::map<int, hipGraphExec_t> g_traj, g_sweep;  // captured per step count
  std::string err;
  std::vector<double> stat_pk, stat_bias, stat_nbar;
};

#define HIPCHK(ctx, call)                                                   \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      (ctx)->err = std::string(#call) + ": " + hipGetErrorString(e_);       \
      return HMC_EDEVICE;                                                   \
    }                                                                       \
  } while (0)

namespace hmc {
int32_t record_free_error(int32_t st, const char* why) {
  g_err = why;
  return st;
}
}  // namespace hmc

static hmc_status fail(hmc_ctx* ctx, hmc_status st, const std::string& why) {
  if (ctx) ctx->err = why;
  g_err = why;
  return st;
}

static hmc_status check_launch(hmc_ctx* ctx) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ctx, HMC_EDEVICE, std::string("launch: ") + hipGetErrorString(e));
  return HMC_OK;
}

// ------------------------------------------------------------------ pass sequences
namespace {

hipEvent_t ev_get(hmc_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// events around one pass launch when timing is on (kind: see hmc_timing)
struct Timed {
  hmc_ctx* c;
  int kind;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(hmc_ctx* c_, int kind_, hipStream_t s) : c(c_), kind(kind_) {
    if (!c->timing || !(c->timing_mask & (1 << kind))) return;
    if (c->timing_seen[kind]++ % c->timing_stride != 0) return;
    a = ev_get(c);
    b = ev_get(c);
    if (a) (void)hipEventRecord(a, s);
  }
  void done(hipStream_t s) {
    if (!a || !b) return;
    (void)hipEventRecord(b, s);
    c->ev_used.push_back({kind, {a, b}});
  }
};

struct Seq {
  hmc_ctx* c;
  const ChainDev* d;
  int nch;
  const int* tot;
  hipStream_t s;
  int un;  // N shared by all chains, or 0
  // calls f(descriptors, chains, tile totals, uniform N, grid) once for the whole
  // batch, or once per size group when the class runs grouped
  template <class F>
  void each(int cls, F f) {
    if (un == 0 && c->grouped[cls] && !c->groups.empty()) {
      for (auto& g : c->groups) f(g.d, g.nch, g.total, g.n, 0);
    } else {
      f(d, nch, tot, un, c->grid[cls]);
    }
  }
  void x(int mode, float kick, float drift, int flags) {
    Timed tm(c, mode == X_STEP ? 0 : 3, s);
    each(0, [&](const ChainDev* dd, int n, const int* t, int u, int g) {
      launch_xpass(mode, dd, n, t[kTileXY], c->lds_x, XArgs{kick, drift, flags}, c->tw, g, s, u,
                   c->plan[0]);
    });
    tm.done(s);
  }
  void y(int dir, int buf = 0) {
    Timed tm(c, 1, s);
    each(1, [&](const ChainDev* dd, int n, const int* t, int u, int g) {
      launch_ypass(dir, dd, n, t[kTileXY], c->lds_x, c->tw, g, s, u, buf, c->plan[1]);
    });
    tm.done(s);
  }
  void xl(int mode, float kick, float drift) {
    Timed tm(c, 3, s);
    each(0, [&](const ChainDev* dd, int n, const int* t, int u, int g) {
      launch_xpass_learned(mode, dd, n, t[kTileXY], c->lds_x, XArgs{kick, drift, 0}, c->tw, g,
                           s, u);
    });
    tm.done(s);
  }
  void zl(int mode, int flags) {
    Timed tm(c, 3, s);
    each(2, [&](const ChainDev* dd, int n, const int* t, int u, int g) {
      launch_zpass_learned(mode, dd, n, t[kTileZ], c->lds_z, ZArgs{flags, 0, nullptr}, c->tw, g,
                           s, u);
    });
    tm.done(s);
  }
  void z(int mode, int flags, const float* src = nullptr) {
    Timed tm(c, mode == Z_GRAD ? 2 : 3, s);
    each(2, [&](const ChainDev* dd, int n, const int* t, int u, int g) {
      launch_zpass(mode, dd, n, t[kTileZ], c->lds_z, ZArgs{flags, 0, src}, c->tw, g, s, u,
                   c->plan[2]);
    });
    tm.done(s);
  }
  // inverse y transforms, the real-space data force (C2R z, alpha delta - beta,
  // R2C z) and forward y transforms: one fused plane pass for grid sizes that have
  // one (the whole context, or each size group of a batch whose y and real-space
  // passes run one launch per size group), else three passes
  void yz(int zflags) {
    const ZArgs za{zflags, 0, nullptr};
    if (c->plane_pass && un != 0 && plane_pass_supported(un)) {
      Timed tm(c, 2, s);
      launch_yzpass(d, nch, za, c->tw, s, un);
      tm.done(s);
      return;
    }
    bool some = false;
    for (auto& g : c->groups) some |= plane_pass_supported(g.n);
    if (c->plane_pass && un == 0 && c->grouped[1] && c->grouped[2] && some) {
      Timed tm(c, 2, s);
      for (auto& g : c->groups) {
        if (plane_pass_supported(g.n)) {
          launch_yzpass(g.d, g.nch, za, c->tw, s, g.n);
        } else {
          launch_ypass(-1, g.d, g.nch, g.total[kTileXY], c->lds_x, c->tw, 0, s, g.n, 0, c->plan[1]);
          launch_zpass(Z_GRAD, g.d, g.nch, g.total[kTileZ], c->lds_z, za, c->tw, 0, s, g.n,
                       c->plan[2]);
          launch_ypass(+1, g.d, g.nch, g.total[kTileXY], c->lds_x, c->tw, 0, s, g.n, 0, c->plan[1]);
        }
      }
      tm.done(s);
      return;
    }
    y(-1);
    z(Z_GRAD, zflags);
    y(+1);
  }
  // g_hat, delta and the data energy of the current delta_hat
  void gradient(int zflags, int xflags) {
    x(X_INV, 0.f, 0.f, xflags & XF_SCALE);
    yz(zflags);
    x(X_FWD, 0.f, 0.f, xflags);
  }
};

Seq seq_all(hmc_ctx* c) {
  return Seq{c, c->d_all, (int)c->ch.size(), c->total, c->stream, c->uniform_n};
}

}  // namespace

static hmc_status refresh_gradient(hmc_ctx* c, bool write_dr) {
  Seq q = seq_all(c);
  q.gradient(ZF_DATA | (write_dr ? ZF_WRITE_DR : 0), 0);
  launch_reduce_slot(c->d_all, (int)c->ch.size(), kPartDat, kDcur, kTileZ, c->stream);
  return check_launch(c);
}

static hmc_status upload_desc(hmc_ctx* c) {
  std::vector<ChainDev> all(c->ch.size());
  for (size_t i = 0; i < c->ch.size(); ++i) all[i] = c->ch[i].dev;
  HIPCHK(c, hipMemcpyAsync(c->d_all, all.data(), all.size() * sizeof(ChainDev),
                           hipMemcpyHostToDevice, c->stream));
  for (auto& k : c->ch) {
    ChainDev s = k.dev;
    for (int j = 0; j < kTileClasses; ++j) s.tb[j] = 0;
    HIPCHK(c, hipMemcpyAsync(k.solo, &s, sizeof(ChainDev), hipMemcpyHostToDevice, c->stream));
  }
  for (auto& g : c->groups) {
    std::vector<ChainDev> gd;
    int base[kTileClasses] = {0, 0, 0, 0};
    for (int i : g.members) {
      ChainDev s = c->ch[i].dev;
      for (int j = 0; j < kTileClasses; ++j) {
        s.tb[j] = base[j];
        base[j] += s.nt[j];
      }
      gd.push_back(s);
    }
    HIPCHK(c, hipMemcpyAsync(g.d, gd.data(), gd.size() * sizeof(ChainDev), hipMemcpyHostToDevice,
                             c->stream));
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HMC_OK;
}

// host -> device parameter block of one chain
static hmc_status push_params(hmc_ctx* c, Chain& k) {
  HIPCHK(c, hipMemcpyAsync(k.dev.P, k.hp.data(), kPSize * sizeof(double), hipMemcpyHostToDevice,
                           c->stream));
  return HMC_OK;
}
static hmc_status pull_params(hmc_ctx* c) {
  for (auto& k : c->ch)
    HIPCHK(c, hipMemcpyAsync(k.hp.data(), k.dev.P, kPSize * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HMC_OK;
}

// recompute alpha, beta, mean(alpha), shell tables for all chains
static hmc_status refresh_coefficients(hmc_ctx* c) {
  const int nch = (int)c->ch.size();
  launch_coeff(c->d_all, nch, c->total[kTileR], c->stream);
  launch_reduce_slot(c->d_all, nch, kPartAlpha, kAbar, kTileR, c->stream, true);
  launch_tables(c->d_all, nch, c->stream);
  return check_launch(c);
}

static hmc_status run_trajectory(hmc_ctx* c);
static hmc_status run_sweep(hmc_ctx* c);

// Capture `body` once on the library's side stream and replay the graph; the
// side stream is ordered after and before the caller's stream with events.
// leapfrog steps of a trajectory / sweep: n_leapfrog, or with tau_mode a uniform
// draw from 1..n_leapfrog (the paper's uniformly drawn pseudo-time tau = n eps)
// from Philox stream 10 of the first chain at the trajectory / sweep index
static int steps_of(hmc_ctx* c, uint64_t index) {
  if (!c->tau_mode) return c->nsteps;
  const hmc_config& f = c->ch[0].cfg;
  const hmcrng::U4 w = hmcrng::block(f.seed, f.chain_id, hmcrng::kTau, (uint32_t)index, 0, 0);
  const int n = 1 + (int)(hmcrng::uniform(w.w[0]) * c->nsteps);
  return n > c->nsteps ? c->nsteps : n;
}

static hmc_status run_graph(hmc_ctx* c, hipGraphExec_t* exec, hmc_status (*body)(hmc_ctx*)) {
  if (!c->gstream) {
    HIPCHK(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev_a, hipEventDisableTiming));
    HIPCHK(c, hipEventCreateWithFlags(&c->gev_b, hipEventDisableTiming));
  }
  if (!*exec) {
    hipStream_t saved = c->stream;
    const bool timing = c->timing;
    c->stream = c->gstream;
    c->timing = false;
    hipError_t e = hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal);
    hmc_status st = e == hipSuccess ? body(c) : HMC_EDEVICE;
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(c->gstream, &g);
    c->stream = saved;
    c->timing = timing;
    if (e != hipSuccess || e2 != hipSuccess || st != HMC_OK || !g) {
      if (g) (void)hipGraphDestroy(g);
      return fail(c, HMC_EDEVICE, std::string("graph capture failed: ") +
                                      hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      *exec = nullptr;
      return fail(c, HMC_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
  }
  HIPCHK(c, hipEventRecord(c->gev_a, c->stream));
  HIPCHK(c, hipStreamWaitEvent(c->gstream, c->gev_a, 0));
  HIPCHK(c, hipGraphLaunch(*exec, c->gstream));
  HIPCHK(c, hipEventRecord(c->gev_b, c->gstream));
  HIPCHK(c, hipStreamWaitEvent(c->stream, c->gev_b, 0));
  return HMC_OK;
}

extern "C" {

size_t hmc_workspace_bytes(const hmc_config* cfg) {
  std::string why;
  if (!valid_cfg(cfg, &why)) return 0;
  return layout(*cfg).total;
}

const char* hmc_last_error(const hmc_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_err.c_str();
}

void hmc_destroy(hmc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& u : ctx->ev_used) {
    (void)hipEventDestroy(u.second.first);
    (void)hipEventDestroy(u.second.second);
  }
  for (auto e : ctx->ev_pool) (void)hipEventDestroy(e);
  for (auto& g : ctx->g_traj) (void)hipGraphExecDestroy(g.second);
  for (auto& g : ctx->g_sweep) (void)hipGraphExecDestroy(g.second);
  if (ctx->gev_a) (void)hipEventDestroy(ctx->gev_a);
  if (ctx->gev_b) (void)hipEventDestroy(ctx->gev_b);
  if (ctx->gstream) (void)hipStreamDestroy(ctx->gstream);
  if (ctx->d_draw) (void)hipFree(ctx->d_draw);
  for (auto& k : ctx->ch) {
    (void)hipFree(k.dev.P);
    (void)hipFree(k.dev.tf);
    (void)hipFree(k.dev.td);
    (void)hipFree(k.solo);
  }
  (void)hipFree(ctx->d_all);
  for (auto& g : ctx->groups) (void)hipFree(g.d);
  (void)hipFree(ctx->tw);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

hmc_status hmc_init_batch(const hmc_config* cfg, const hmc_buffers* buf, int32_t n_chains,
                          const double* bias, const double* nbar, const double* pk, void* stream,
                          hmc_ctx** out) {
  if (!out) return fail(nullptr, HMC_EINVAL, "null output pointer");
  *out = nullptr;
  if (n_chains < 1 || !cfg || !buf || !bias || !nbar || !pk)
    return fail(nullptr, HMC_EINVAL, "null argument or n_chains < 1");
  std::string why;
  for (int i = 0; i < n_chains; ++i) {
    if (!valid_cfg(&cfg[i], &why)) return fail(nullptr, HMC_EINVAL, why);
    if (cfg[i].n_leapfrog != cfg[0].n_leapfrog)
      return fail(nullptr, HMC_EINVAL, "all chains of a batch need the same n_leapfrog");
    if (cfg[i].tau_mode != cfg[0].tau_mode)
      return fail(nullptr, HMC_EINVAL, "all chains of a batch need the same tau_mode");
    const hmc_buffers& b = buf[i];
    if (!b.R || !b.counts || !b.delta_k || !b.mom_k || !b.grad_k || !b.delta_r || !b.alpha ||
        !b.beta || !b.work)
      return fail(nullptr, HMC_EINVAL, "null buffer");
    if (b.work_bytes < layout(cfg[i]).total)
      return fail(nullptr, HMC_ENOMEM, "workspace smaller than hmc_workspace_bytes()");
  }
  hmc_ctx* c = new hmc_ctx();
  c->stream = (hipStream_t)stream;
  c->nsteps = c->cur_steps = cfg[0].n_leapfrog;
  c->tau_mode = cfg[0].tau_mode;
  c->ch.resize(n_chains);
  auto bail = [&](hmc_status st) {
    g_err = c->err;
    hmc_destroy(c);
    return st;
  };
  // twiddle tables, computed in float64
  {
    std::vector<float2> tw(kTwTotal);
    const int lens[] = {4, 8, 16, 32, 64, 96, 128, 192, 256};
    for (int L : lens)
      for (int i = 0; i < L; ++i) {
        const double a = -2.0 * M_PI * (double)i / (double)L;
        tw[tw_offset(L) + i] = make_float2((float)std::cos(a), (float)std::sin(a));
      }
    const hipError_t e = hipMalloc(&c->tw, kTwTotal * sizeof(float2));
    if (e != hipSuccess) {
      c->err = std::string("hipMalloc twiddles: ") + hipGetErrorString(e);
      return bail(HMC_EDEVICE);
    }
    if (hipMemcpy(c->tw, tw.data(), kTwTotal * sizeof(float2), hipMemcpyHostToDevice) !=
        hipSuccess) {
      c->err = "twiddle upload";
      return bail(HMC_EDEVICE);
    }
  }
  if (hipMalloc(&c->d_draw, 64) != hipSuccess) {
    c->err = "hipMalloc draw counter";
    return bail(HMC_EDEVICE);
  }
  if (hipHostMalloc((void**)&c->pinned, 64 * sizeof(double), 0) != hipSuccess) {
    c->err = "hipHostMalloc";
    return bail(HMC_EDEVICE);
  }
  int boff = 0, soff = 0;
  int base[kTileClasses] = {0, 0, 0, 0};
  for (int i = 0; i < n_chains; ++i) {
    Chain& k = c->ch[i];
    k.cfg = cfg[i];
    k.buf = buf[i];
    const int n = k.cfg.n;
    const WsLayout L = layout(k.cfg);
    ChainDev& d = k.dev;
    memset(&d, 0, sizeof(d));
    d.n = n;
    d.h = n / 2 + 1;
    d.nb = k.cfg.n_bins;
    d.nsub = k.cfg.n_sub;
    d.nv = (long long)n * n * n;
    d.nh = (long long)n * n * (n / 2 + 1);
    d.norm = (float)(1.0 / std::sqrt((double)d.nv));
    d.eps = (float)k.cfg.eps;
    d.seed = k.cfg.seed;
    d.chain = k.cfg.chain_id;
    d.fixed_mask = k.cfg.fixed_bias_mask;
    d.alpha_prior = k.cfg.alpha_prior;
    d.box = k.cfg.box;
    for (int j = 0; j < kTileClasses; ++j) {
      d.nt[j] = tiles_of(j, n);
      d.tb[j] = base[j];
      base[j] += d.nt[j];
    }
    d.maxtiles = L.maxtiles;
    d.draw = c->d_draw;
    d.R = k.buf.R;
    d.counts = k.buf.counts;
    d.growth = k.buf.growth;
    d.dk = (float2*)k.buf.delta_k;
    d.pk = (float2*)k.buf.mom_k;
    d.gk = (float2*)k.buf.grad_k;
    d.dr = k.buf.delta_r;
    d.alpha = k.buf.alpha;
    d.beta = k.buf.beta;
    char* w = (char*)k.buf.work;
    d.T = (float2*)(w + L.T);
    d.bdk = (float2*)(w + L.bdk);
    d.bgk = (float2*)(w + L.bgk);
    d.drn = (float*)(w + L.drn);
    d.part = (double*)(w + L.part);
    d.shpart = (double*)(w + L.shpart);
    d.mpart = (double*)(w + L.mpart);
    d.T2 = (float2*)(w + L.T2);
    d.T3 = (float2*)(w + L.T3);
    d.shat = (float2*)(w + L.shat);
    d.smass = (float*)(w + L.smass);
    d.lut = (signed char*)(w + L.lut);
    d.obs = (unsigned long long*)(w + L.obs);
    if (hipMalloc(&d.P, kPSize * sizeof(double)) != hipSuccess ||
        hipMalloc(&d.tf, kTSize * sizeof(float)) != hipSuccess ||
        hipMalloc(&d.td, kDSize * sizeof(double)) != hipSuccess ||
        hipMalloc(&k.solo, sizeof(ChainDev)) != hipSuccess) {
      c->err = "hipMalloc parameter block";
      return bail(HMC_EDEVICE);
    }
    k.hp.assign(kPSize, 0.0);
    const double lamf = std::pow((double)n, 3) / std::pow(k.cfg.box, 3);
    const double bound = k.cfg.rj_log_bound > 0 ? k.cfg.rj_log_bound : 10.0;
    for (int m = 0; m < d.nb; ++m) {
      const double lam = pk[soff + m] * lamf;
      if (!(lam > 0) || !std::isfinite(lam)) {
        c->err = "pk must be positive and finite";
        return bail(HMC_EINVAL);
      }
      k.hp[kLam + m] = lam;
      k.hp[kLo + m] = std::log(lam) - bound;
      k.hp[kHi + m] = std::log(lam) + bound;
    }
    for (int l = 0; l < d.nsub; ++l) {
      k.hp[kBias + l] = bias[boff + l];
      k.hp[kNbar + l] = nbar[boff + l];
    }
    boff += d.nsub;
    soff += d.nb;
    c->max_nb = std::max(c->max_nb, d.nb);
    c->max_sub = std::max(c->max_sub, d.nsub);
    c->lds_x = std::max(c->lds_x, xpass_lds_bytes(n));
    c->lds_z = std::max(c->lds_z, zpass_lds_bytes(n));
  }
  for (int j = 0; j < kTileClasses; ++j) c->total[j] = base[j];
  c->uniform_n = c->ch[0].cfg.n;
  for (auto& k : c->ch)
    if (k.cfg.n != c->uniform_n) c->uniform_n = 0;
  if (hipMalloc(&c->d_all, n_chains * sizeof(ChainDev)) != hipSuccess) {
    c->err = "hipMalloc descriptors";
    return bail(HMC_EDEVICE);
  }
  if (c->uniform_n == 0) {
    for (int i = 0; i < n_chains; ++i) {
      const int n = c->ch[i].cfg.n;
      auto it = std::find_if(c->groups.begin(), c->groups.end(),
                             [n](const hmc_ctx::Group& g) { return g.n == n; });
      if (it == c->groups.end()) {
        c->groups.emplace_back();
        it = c->groups.end() - 1;
        it->n = n;
      }
      it->members.push_back(i);
      it->nch += 1;
      for (int j = 0; j < kTileClasses; ++j) it->total[j] += c->ch[i].dev.nt[j];
    }
    for (auto& g : c->groups)
      if (hipMalloc(&g.d, g.nch * sizeof(ChainDev)) != hipSuccess) {
        c->err = "hipMalloc group descriptors";
        return bail(HMC_EDEVICE);
      }
  }
  hmc_status st;
  for (auto& k : c->ch)
    if ((st = push_params(c, k)) != HMC_OK) return bail(st);
  if ((st = upload_desc(c)) != HMC_OK) return bail(st);
  const int nch = n_chains;
  for (auto& k : c->ch) launch_shell_lut(k.solo, k.cfg.n, c->stream);
  // survey support, static data sums, mode counts, coefficients, tables, gradient of
  // the initial state
  launch_obs_mask(c->d_all, nch, c->total[kTileR], c->stream);
  launch_static_moments(c->d_all, nch, c->total[kTileR], c->stream);
  launch_colsum(c->d_all, nch, 3 * c->max_sub, 1, kTileR, kS0, 1, c->stream);
  launch_shell_power(c->d_all, nch, c->total[kTileK], c->stream, 1);
  launch_colsum(c->d_all, nch, c->max_nb, 1, kTileK, kNmodes, 0, c->stream);
  launch_colsum(c->d_all, nch, c->max_nb, 0, kTileK, kSigma, 0, c->stream);
  if ((st = refresh_coefficients(c)) != HMC_OK) return bail(st);
  if ((st = refresh_gradient(c, true)) != HMC_OK) return bail(st);
  if ((st = pull_params(c)) != HMC_OK) return bail(st);
  for (auto& k : c->ch)
    for (int m = 0; m < k.dev.nb; ++m)
      if (k.hp[kNmodes + m] <= 0) {
        c->err = "a k-shell has no modes; use fewer bins";
        return bail(HMC_EINVAL);
      }
  // the Nbar^l conditional needs observed voxels (R^l > 0) in every subsample
  for (auto& k : c->ch)
    for (int l = 0; l < k.dev.nsub; ++l)
      if (k.hp[kNobs + l] <= 0) {
        c->err = "a subsample has no voxel with R > 0";
        return bail(HMC_EINVAL);
      }
  *out = c;
  return HMC_OK;
}

hmc_status hmc_init(const hmc_config* cfg, const hmc_buffers* buf, const double* bias,
                    const double* nbar, const double* pk, void* stream, hmc_ctx** out) {
  return hmc_init_batch(cfg, buf, 1, bias, nbar, pk, stream, out);
}

// one density trajectory for every chain; results stay on the device
// one density trajectory for every chain (draw index from the device counter);
// no host synchronisation, so it can be captured in a graph
// density trajectory with the learned mass (see the learned-mass passes in
// kernels.hip); the plain gradient cache is refreshed after the Metropolis test
static hmc_status run_trajectory_learned(hmc_ctx* c) {
  Seq q = seq_all(c);
  const int nch = (int)c->ch.size();
  auto force = [&](int zflags) {
    q.y(-1, 0);
    q.y(-1, 2);
    q.zl(LZ_FORCE, zflags);
    launch_reduce_slot(c->d_all, nch, kPartAux, kGbar, kTileZ, c->stream, true);
    q.y(+1, 0);
  };
  q.z(Z_NOISE, 0);
  q.y(+1);
  q.xl(L_START, 0.f, 0.f);
  launch_reduce_slot(c->d_all, nch, kPartKin, kK0, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartPri, kPi0, kTileXY, c->stream);
  force(0);
  q.xl(L_KICK, 0.5f, 0.f);
  for (int s = 1; s <= c->cur_steps; ++s) {
    const bool last = s == c->cur_steps;
    q.y(-1, 1);
    q.zl(LZ_VEL, 0);
    q.y(+1, 1);
    q.xl(L_DRIFT, 0.f, 1.f);
    force(last ? (ZF_WRITE_DRN | ZF_DATA) : 0);
    q.xl(last ? L_KICK_LAST : L_KICK, last ? 0.5f : 1.f, 0.f);
  }
  launch_reduce_slot(c->d_all, nch, kPartKin, kK1, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartPri, kPi1, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartDat, kD1, kTileZ, c->stream);
  launch_accept(c->d_all, nch, c->stream);
  launch_commit(C_HMC, c->d_all, nch, c->total[kTileK], c->total[kTileR], c->stream);
  return refresh_gradient(c, false);
}

static hmc_status run_trajectory(hmc_ctx* c) {
  if (c->learned) return run_trajectory_learned(c);
  Seq q = seq_all(c);
  const int nch = (int)c->ch.size();
  q.z(Z_NOISE, 0);
  q.y(+1);
  q.x(X_START, 0.5f, 1.f, 0);
  launch_reduce_slot(c->d_all, nch, kPartKin, kK0, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartPri, kPi0, kTileXY, c->stream);
  for (int s = 1; s < c->cur_steps; ++s) {
    q.yz(0);
    q.x(X_STEP, 1.f, 1.f, 0);
  }
  q.yz(ZF_WRITE_DRN | ZF_DATA);
  q.x(X_END, 0.5f, 0.f, 0);
  launch_reduce_slot(c->d_all, nch, kPartKin, kK1, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartPri, kPi1, kTileXY, c->stream);
  launch_reduce_slot(c->d_all, nch, kPartDat, kD1, kTileZ, c->stream);
  launch_accept(c->d_all, nch, c->stream);
  launch_commit(C_HMC, c->d_all, nch, c->total[kTileK], c->total[kTileR], c->stream);
  return check_launch(c);
}

hmc_status leapfrog_trajectory(hmc_ctx* c, uint64_t traj_index, double* dH, int32_t* accepted) {
  if (!c) return fail(nullptr, HMC_EINVAL, "null context");
  if (c->mass_mixed)
    return fail(c, HMC_EUNSUPPORTED, "learned mass set on some chains of the context only");
  launch_set_draw(c->d_draw, (uint32_t)traj_index, c->stream);
  c->cur_steps = steps_of(c, traj_index);
  hmc_status st = c->use_graph ? run_graph(c, &c->g_traj[c->cur_steps], run_trajectory)
                               : run_trajectory(c);
  if (st != HMC_OK) return st;
  if ((st = pull_params(c)) != HMC_OK) return st;
  bool numeric = false;
  for (size_t i = 0; i < c->ch.size(); ++i) {
    if (dH) dH[i] = c->ch[i].hp[kDH];
    if (accepted) accepted[i] = c->ch[i].hp[kAcc] != 0.0;
    numeric |= c->ch[i].hp[kStatus] == 1.0;
  }
  return numeric ? fail(c, HMC_ENUMERIC, "non-finite energy; trajectory rejected") : HMC_OK;
}

hmc_status leapfrog_trajectory_async(hmc_ctx* c, uint64_t traj_index, double* dH_dev,
                                     int32_t* accepted_dev) {
  if (!c || !dH_dev || !accepted_dev) return fail(c, HMC_EINVAL, "bad argument");
  if (c->mass_mixed)
    return fail(c, HMC_EUNSUPPORTED, "learned mass set on some chains of the context only");
  launch_set_draw(c->d_draw, (uint32_t)traj_index, c->stream);
  c->cur_steps = steps_of(c, traj_index);
  hmc_status st = c->use_graph ? run_graph(c, &c->g_traj[c->cur_steps], run_trajectory)
                               : run_trajectory(c);
  if (st != HMC_OK) return st;
  launch_export(c->d_all, (int)c->ch.size(), 0, dH_dev, accepted_dev, c->stream);
  return check_launch(c);
}

hmc_status hamiltonian(hmc_ctx* c, int32_t chain, double* out) {
  if (!c || !out || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  launch_energy_k(k.solo, 1, k.dev.nt[kTileK], c->stream);
  launch_reduce_slot(k.solo, 1, kPartKin, kHK, kTileK, c->stream);
  launch_reduce_slot(k.solo, 1, kPartPri, kHP, kTileK, c->stream);
  launch_energy_r(k.solo, 1, k.dev.nt[kTileR], c->stream);
  launch_reduce_slot(k.solo, 1, kPartDat, kHD, kTileR, c->stream);
  hmc_status st = check_launch(c);
  if (st != HMC_OK) return st;
  if ((st = pull_params(c)) != HMC_OK) return st;
  out[0] = k.hp[kHK];
  out[1] = k.hp[kHP];
  out[2] = k.hp[kHD];
  return HMC_OK;
}

hmc_status shell_power(hmc_ctx* c, int32_t chain, double* sigma, int64_t* n_modes) {
  if (!c || !sigma || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  launch_shell_power(k.solo, 1, k.dev.nt[kTileK], c->stream);
  launch_colsum(k.solo, 1, k.dev.nb, 0, kTileK, kSigma, 0, c->stream);
  hmc_status st = check_launch(c);
  if (st != HMC_OK) return st;
  if ((st = pull_params(c)) != HMC_OK) return st;
  for (int m = 0; m < k.dev.nb; ++m) {
    sigma[m] = k.hp[kSigma + m];
    if (n_modes) n_modes[m] = (int64_t)k.hp[kNmodes + m];
  }
  return HMC_OK;
}

// the device part of one block sweep for every chain (no host synchronisation)
static hmc_status run_sweep(hmc_ctx* c) {
  const int nch = (int)c->ch.size();
  hmc_status st = run_trajectory(c);
  if (st != HMC_OK) return st;
  // P | delta
  launch_shell_power(c->d_all, nch, c->total[kTileK], c->stream);
  launch_colsum(c->d_all, nch, c->max_nb, 0, kTileK, kSigma, 0, c->stream);
  launch_draw_power(c->d_all, nch, c->stream);
  launch_tables(c->d_all, nch, c->stream);
  // joint (P, delta) move for chains that ask for it (all or none in a batch)
  bool any_rj = false;
  for (auto& k : c->ch) any_rj |= k.cfg.rj_move != 0;
  if (any_rj) {
    Seq q = seq_all(c);
    // dU at the start: per-shell Re(conj(delta_hat) g_hat) at the current state.
    // grad_k holds g_hat of delta_hat here (the trajectory's last gradient, or the
    // restored one of its start; the P draw does not change alpha, beta), so one
    // k-space pass over the stored arrays gives it.
    launch_shell_dot(c->d_all, nch, c->total[kTileK], c->stream);
    launch_rj(RJ_BEGIN, c->d_all, nch, c->max_nb, c->stream, kTileK);
    for (int i = 0; i < c->cur_steps; ++i) {
      const bool last = i == c->cur_steps - 1;
      q.gradient(last ? (ZF_WRITE_DRN | ZF_DATA) : 0,
                 XF_SCALE | XF_DOT | (last ? XF_OUT_ALT : XF_NOSTORE));
      if (!last) {
        launch_rj(RJ_STEP, c->d_all, nch, c->max_nb, c->stream);
      } else {
        launch_reduce_slot(c->d_all, nch, kPartDat, kD1, kTileZ, c->stream);
        launch_rj(RJ_END, c->d_all, nch, c->max_nb, c->stream);
      }
    }
    launch_commit(C_RJ, c->d_all, nch, c->total[kTileK], c->total[kTileR], c->stream);
    launch_tables(c->d_all, nch, c->stream);
  }
  // Nbar | delta, b and b | delta, Nbar
  launch_moments(c->d_all, nch, c->total[kTileR], c->stream);
  launch_colsum(c->d_all, nch, 3 * c->max_sub, 1, kTileR, kS1, 1, c->stream);
  launch_draw_nbar_bias(c->d_all, nch, c->stream);
  // alpha, beta, mass and gradient for the new parameters
  if ((st = refresh_coefficients(c)) != HMC_OK) return st;
  return refresh_gradient(c, false);
}

hmc_status gibbs_sweep(hmc_ctx* c, uint64_t sweep_index, hmc_sweep_stats* out) {
  if (!c) return fail(nullptr, HMC_EINVAL, "null context");
  if (c->mass_mixed)
    return fail(c, HMC_EUNSUPPORTED, "learned mass set on some chains of the context only");
  launch_set_draw(c->d_draw, (uint32_t)sweep_index, c->stream);
  c->cur_steps = steps_of(c, sweep_index);
  hmc_status st = c->use_graph ? run_graph(c, &c->g_sweep[c->cur_steps], run_sweep) : run_sweep(c);
  if (st != HMC_OK) return st;
  if ((st = pull_params(c)) != HMC_OK) return st;
  c->stat_pk.clear();
  c->stat_bias.clear();
  c->stat_nbar.clear();
  bool bad = false;
  for (auto& k : c->ch) {
    const double f = std::pow(k.cfg.box, 3) / std::pow((double)k.cfg.n, 3);
    for (int m = 0; m < k.dev.nb; ++m) c->stat_pk.push_back(k.hp[kLam + m] * f);
    for (int l = 0; l < k.dev.nsub; ++l) {
      c->stat_bias.push_back(k.hp[kBias + l]);
      c->stat_nbar.push_back(k.hp[kNbar + l]);
    }
    bad |= k.hp[kStatus] != 0.0;
  }
  if (out) {
    size_t po = 0, bo = 0;
    for (size_t i = 0; i < c->ch.size(); ++i) {
      const Chain& k = c->ch[i];
      out[i].dH = k.hp[kDH];
      out[i].accepted = k.hp[kAcc] != 0.0;
      out[i].rj_dH = k.cfg.rj_move ? k.hp[kRjDH] : 0.0;
      out[i].rj_accepted = k.cfg.rj_move ? k.hp[kRjAcc] != 0.0 : 0;
      out[i].rj_wall_hits = k.cfg.rj_move ? (int32_t)k.hp[kRjHits] : 0;
      out[i].pk = c->stat_pk.data() + po;
      out[i].bias = c->stat_bias.data() + bo;
      out[i].nbar = c->stat_nbar.data() + bo;
      po += k.dev.nb;
      bo += k.dev.nsub;
    }
  }
  return bad ? fail(c, HMC_ENUMERIC, "a draw or an energy was not finite") : HMC_OK;
}

size_t hmc_sweep_record_doubles(const hmc_ctx* c) {
  if (!c) return 0;
  size_t n = 0;
  for (auto& k : c->ch) n += kRecHead + k.dev.nb + 2 * k.dev.nsub;
  return n;
}

hmc_status gibbs_sweep_async(hmc_ctx* c, uint64_t sweep_index, double* stats_dev) {
  if (!c || !stats_dev) return fail(c, HMC_EINVAL, "bad argument");
  if (c->mass_mixed)
    return fail(c, HMC_EUNSUPPORTED, "learned mass set on some chains of the context only");
  launch_set_draw(c->d_draw, (uint32_t)sweep_index, c->stream);
  c->cur_steps = steps_of(c, sweep_index);
  hmc_status st = c->use_graph ? run_graph(c, &c->g_sweep[c->cur_steps], run_sweep) : run_sweep(c);
  if (st != HMC_OK) return st;
  launch_export(c->d_all, (int)c->ch.size(), 1, stats_dev, nullptr, c->stream);
  return check_launch(c);
}

hmc_status hmc_set_state(hmc_ctx* c, int32_t chain, const float* delta_r_dev) {
  if (!c || !delta_r_dev || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  const int tz = k.dev.nt[kTileZ], tx = k.dev.nt[kTileXY];
  launch_zpass(Z_R2C, k.solo, 1, tz, c->lds_z, ZArgs{0, 0, delta_r_dev}, c->tw, 0, c->stream, k.cfg.n);
  launch_ypass(+1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_xpass(X_FWD, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, XF_OUT_DK}, c->tw, 0, c->stream, k.cfg.n);
  // gradient, real field and data energy of the new state
  launch_xpass(X_INV, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, 0}, c->tw, 0, c->stream, k.cfg.n);
  launch_ypass(-1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_zpass(Z_GRAD, k.solo, 1, tz, c->lds_z, ZArgs{ZF_DATA | ZF_WRITE_DR, 0, nullptr}, c->tw,
               0, c->stream, k.cfg.n);
  launch_ypass(+1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_xpass(X_FWD, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, 0}, c->tw, 0, c->stream, k.cfg.n);
  launch_reduce_slot(k.solo, 1, kPartDat, kDcur, kTileZ, c->stream);
  return check_launch(c);
}

hmc_status hmc_field_moments(hmc_ctx* c, int32_t chain, double* mean_dev, double* m2_dev,
                             int64_t count) {
  if (!c || !mean_dev || !m2_dev || chain < 0 || chain >= (int)c->ch.size() || count < 1)
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  launch_field_moments(k.buf.delta_r, mean_dev, m2_dev, k.dev.nv, (long long)count, c->stream);
  return check_launch(c);
}

hmc_status hmc_warm_start(hmc_ctx* c, int32_t chain, const float* mu_dev,
                          const float* logvar_dev, uint64_t draw_index) {
  if (!c || !mu_dev || !logvar_dev || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  const int tz = k.dev.nt[kTileZ], tx = k.dev.nt[kTileXY], tr = k.dev.nt[kTileR];
  // prior draw xi = F^-1(sqrt(lambda_k) F w) into the proposal buffer
  launch_set_draw(c->d_draw, (uint32_t)draw_index, c->stream);
  launch_zpass(Z_NOISE, k.solo, 1, tz, c->lds_z, ZArgs{ZF_WARM, 0, nullptr}, c->tw, 0, c->stream,
               k.cfg.n);
  launch_ypass(+1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_xpass(X_FWD, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, XF_OUT_DK}, c->tw, 0, c->stream,
               k.cfg.n);
  launch_xpass(X_INV, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, XF_PRIOR}, c->tw, 0, c->stream,
               k.cfg.n);
  launch_ypass(-1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_zpass(Z_C2R, k.solo, 1, tz, c->lds_z, ZArgs{ZF_WRITE_DRN, 0, nullptr}, c->tw, 0,
               c->stream, k.cfg.n);
  launch_warm_combine(k.solo, tr, mu_dev, logvar_dev, c->stream);
  hmc_status st = check_launch(c);
  if (st != HMC_OK) return st;
  return hmc_set_state(c, chain, k.dev.drn);
}

hmc_status hmc_set_params(hmc_ctx* c, int32_t chain, const double* pk, const double* bias,
                          const double* nbar) {
  if (!c || chain < 0 || chain >= (int)c->ch.size()) return fail(c, HMC_EINVAL, "bad argument");
  hmc_status st = pull_params(c);
  if (st != HMC_OK) return st;
  Chain& k = c->ch[chain];
  const double lamf = std::pow((double)k.cfg.n, 3) / std::pow(k.cfg.box, 3);
  if (pk)
    for (int m = 0; m < k.dev.nb; ++m) {
      if (!(pk[m] > 0)) return fail(c, HMC_EINVAL, "pk must be positive");
      k.hp[kLam + m] = pk[m] * lamf;
    }
  for (int l = 0; l < k.dev.nsub; ++l) {
    if (bias) k.hp[kBias + l] = bias[l];
    if (nbar) k.hp[kNbar + l] = nbar[l];
  }
  if ((st = push_params(c, k)) != HMC_OK) return st;
  if ((st = refresh_coefficients(c)) != HMC_OK) return st;
  return refresh_gradient(c, true);
}

hmc_status hmc_set_coefficients(hmc_ctx* c, int32_t chain, const float* alpha_dev,
                                const float* beta_dev) {
  if (!c || !alpha_dev || !beta_dev || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  const size_t bytes = (size_t)k.dev.nv * sizeof(float);
  HIPCHK(c, hipMemcpyAsync(k.buf.alpha, alpha_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(k.buf.beta, beta_dev, bytes, hipMemcpyDeviceToDevice, c->stream));
  // mean(alpha) from the new field: reuse the coefficient partial slot via the
  // real-space energy kernel layout (sum of alpha per tile)
  launch_alpha_sum(k.solo, 1, k.dev.nt[kTileR], c->stream);
  launch_reduce_slot(k.solo, 1, kPartAlpha, kAbar, kTileR, c->stream, true);
  launch_tables(k.solo, 1, c->stream);
  return refresh_gradient(c, true);
}

hmc_status hmc_set_step(hmc_ctx* c, int32_t chain, double eps) {
  if (!c || chain < 0 || chain >= (int)c->ch.size() || !(eps > 0) || !std::isfinite(eps))
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  k.cfg.eps = eps;
  k.dev.eps = (float)eps;
  hmc_status st = upload_desc(c);
  if (st != HMC_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HMC_OK;
}

hmc_status hmc_get_params(hmc_ctx* c, int32_t chain, double* pk, double* bias, double* nbar) {
  if (!c || chain < 0 || chain >= (int)c->ch.size()) return fail(c, HMC_EINVAL, "bad argument");
  hmc_status st = pull_params(c);
  if (st != HMC_OK) return st;
  Chain& k = c->ch[chain];
  const double f = std::pow(k.cfg.box, 3) / std::pow((double)k.cfg.n, 3);
  if (pk)
    for (int m = 0; m < k.dev.nb; ++m) pk[m] = k.hp[kLam + m] * f;
  for (int l = 0; l < k.dev.nsub; ++l) {
    if (bias) bias[l] = k.hp[kBias + l];
    if (nbar) nbar[l] = k.hp[kNbar + l];
  }
  return HMC_OK;
}

hmc_status hmc_shell_index(hmc_ctx* c, int32_t chain, int16_t* out_dev) {
  if (!c || !out_dev || chain < 0 || chain >= (int)c->ch.size())
    return fail(c, HMC_EINVAL, "bad argument");
  Chain& k = c->ch[chain];
  launch_shell_index(k.solo, k.dev.nt[kTileK], out_dev, c->stream);
  hmc_status st = check_launch(c);
  if (st != HMC_OK) return st;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return HMC_OK;
}

hmc_status hmc_use_graph(hmc_ctx* c, int32_t enable) {
  if (!c) return fail(nullptr, HMC_EINVAL, "null context");
  c->use_graph = enable != 0;
  return HMC_OK;
}

static void drop_graphs(hmc_ctx* c) {
  for (auto& g : c->g_traj) (void)hipGraphExecDestroy(g.second);
  for (auto& g : c->g_sweep) (void)hipGraphExecDestroy(g.second);
  c->g_traj.clear();
  c->g_sweep.clear();
}

static int class_tiles(hmc_ctx* c, int cls) { return c->total[cls == 2 ? kTileZ : kTileXY]; }

hmc_status hmc_set_launch(hmc_ctx* c, int32_t cls, int32_t grid) {
  if (!c || cls < 0 || cls > 2 || grid < -1) return fail(c, HMC_EINVAL, "bad argument");
  c->grouped[cls] = grid == -1 && !c->groups.empty();
  c->grid[cls] = grid < 0 || grid >= class_tiles(c, cls) ? 0 : grid;
  drop_graphs(c);
  return HMC_OK;
}

hmc_status hmc_set_plan(hmc_ctx* c, int32_t cls, int32_t plan) {
  if (!c || cls < 0 || cls > 2 || plan < 0 || plan >= kPlanCount)
    return fail(c, HMC_EINVAL, "bad argument");
  c->plan[cls] = plan;
  drop_graphs(c);
  return HMC_OK;
}

hmc_status hmc_set_plane_pass(hmc_ctx* c, int32_t enable) {
  if (!c || (enable != 0 && enable != 1)) return fail(c, HMC_EINVAL, "bad argument");
  c->plane_pass = enable != 0;
  drop_graphs(c);
  return HMC_OK;
}

hmc_status hmc_get_launch(hmc_ctx* c, int32_t* grid, int32_t* plan) {
  if (!c) return fail(nullptr, HMC_EINVAL, "null context");
  for (int cls = 0; cls < 3; ++cls) {
    if (grid) grid[cls] = c->grouped[cls] ? -1 : c->grid[cls];
    if (plan) plan[cls] = c->plan[cls];
  }
  return HMC_OK;
}

// true if some chain's grid size has alternative radix plans
static bool any_plans(const hmc_ctx* c) {
  for (auto& k : c->ch) {
    const int n = k.cfg.n;
    if (n == 64 || n == 128 || n == 192 || n == 256) return true;
  }
  return false;
}

// One launch of the pass class on every chain.  The k-space pass runs with zero
// kick and drift (it rewrites delta_hat and p_hat with their own values); the y
// and real-space passes only touch the intermediate grid, which no call expects
// to survive between calls.
static void tune_launch(hmc_ctx* c, int cls) {
  Seq q = seq_all(c);
  if (cls == 0)
    q.x(X_STEP, 0.f, 0.f, 0);
  else if (cls == 1)
    q.y(-1);
  else
    q.z(Z_GRAD, 0);
}

hmc_status hmc_autotune(hmc_ctx* c, int32_t reps, int32_t* chosen) {
  if (!c || reps < 1) return fail(c, HMC_EINVAL, "bad argument");
  int dev = 0, cus = 0;
  HIPCHK(c, hipGetDevice(&dev));
  HIPCHK(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const bool timing = c->timing;
  c->timing = false;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(c, hipEventCreate(&a));
  HIPCHK(c, hipEventCreate(&b));
  const int mult[] = {0, 2, 3, 4, 5, 6, 8, 12};
  hmc_status st = HMC_OK;
  auto time_class = [&](int cls, float* ms) -> bool {
    tune_launch(c, cls);  // warm-up
    if (hipEventRecord(a, c->stream) != hipSuccess) return false;
    for (int r = 0; r < reps; ++r) tune_launch(c, cls);
    if (hipEventRecord(b, c->stream) != hipSuccess || hipEventSynchronize(b) != hipSuccess)
      return false;
    *ms = 0.f;
    (void)hipEventElapsedTime(ms, a, b);
    return true;
  };
  // batches whose size groups have a fused plane pass run it only when the y and
  // real-space classes launch per size group, so those classes keep that launch
  bool plane_groups = false;
  for (auto& g : c->groups) plane_groups |= plane_pass_supported(g.n);
  plane_groups &= c->plane_pass && c->uniform_n == 0;
  for (int cls = 0; cls < 3 && st == HMC_OK; ++cls) {
    float best = 0.f;
    int best_grid = 0;
    bool best_grouped = false;
    c->plan[cls] = 0;
    // candidates: one launch per size group (batches of several sizes), then one
    // launch over the whole batch with each grid
    const int last = plane_groups && cls > 0 ? 0 : (int)(sizeof(mult) / sizeof(int));
    for (int cand = c->groups.empty() ? 0 : -1; cand < last; ++cand) {
      const bool grp = cand < 0;
      const int grid = grp ? 0 : mult[cand] * cus;
      if (!grp && mult[cand] > 0 && (grid >= class_tiles(c, cls) || grid % 8 != 0)) continue;
      c->grouped[cls] = grp;
      c->grid[cls] = grid;
      float ms = 0.f;
      if (!time_class(cls, &ms)) {
        st = HMC_EDEVICE;
        break;
      }
      if (best == 0.f || ms < best) {
        best = ms;
        best_grid = grid;
        best_grouped = grp;
      }
    }
    c->grid[cls] = best_grid;
    c->grouped[cls] = best_grouped;
    if (chosen) chosen[cls] = best_grouped ? -1 : best_grid;
    // radix plans of the single-size launches at the chosen grid
    if (st == HMC_OK && any_plans(c) && (c->uniform_n != 0 || best_grouped)) {
      int best_plan = 0;
      for (int p = 1; p < kPlanCount; ++p) {
        c->plan[cls] = p;
        float ms = 0.f;
        if (!time_class(cls, &ms)) {
          st = HMC_EDEVICE;
          break;
        }
        if (ms < best) {
          best = ms;
          best_plan = p;
        }
      }
      c->plan[cls] = best_plan;
    }
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  c->timing = timing;
  drop_graphs(c);
  if (st != HMC_OK) return fail(c, st, "autotune: event failure");
  return check_launch(c);
}

hmc_status hmc_timing(hmc_ctx* c, int32_t enable, double* ms, int64_t* launches) {
  if (!c) return fail(nullptr, HMC_EINVAL, "null context");
  if (!c->ev_used.empty()) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto& u : c->ev_used) {
      float t = 0.f;
      HIPCHK(c, hipEventElapsedTime(&t, u.second.first, u.second.second));
      c->t_ms[u.first] += t;
      c->t_n[u.first] += 1;
      c->ev_pool.push_back(u.second.first);
      c->ev_pool.push_back(u.second.second);
    }
    c->ev_used.clear();
  }
  for (int i = 0; i < 4; ++i) {
    if (ms) ms[i] = c->t_ms[i];
    if (launches) launches[i] = c->t_n[i];
  }
  if (enable == 1 || (enable >= 0x10 && enable < 0x10000 && (enable & 0xf0) == 0x10)) {
    for (int i = 0; i < 4; ++i) {
      c->t_ms[i] = 0.0;
      c->t_n[i] = 0;
      c->timing_seen[i] = 0;
    }
    c->timing = true;
    c->timing_mask = enable == 1 ? 0xf : (enable & 0xf);
    c->timing_stride = enable == 1 ? 1 : ((enable >> 8) & 0xff) + 1;
  } else if (enable == 0) {
    c->timing = false;
  }
  return HMC_OK;
}

static hmc_status set_mass_one(hmc_ctx* c, Chain& k, const float* logvar_dev, bool flat) {
  if (logvar_dev == nullptr) {
    k.learned = false;
    k.dev.mass_flat = 0;
    return HMC_OK;
  }
  const int tr = k.dev.nt[kTileR], tz = k.dev.nt[kTileZ], tx = k.dev.nt[kTileXY];
  launch_mass_prep(0, k.solo, tr, logvar_dev, c->stream);
  launch_reduce_slot(k.solo, 1, kPartAux, kLmean, kTileR, c->stream, true);
  launch_mass_prep(1, k.solo, tr, logvar_dev, c->stream);
  // F(D^(1/2)) (unitary, k = 0 entry zeroed) for the mean-removal term of the kick
  launch_zpass(Z_R2C, k.solo, 1, tz, c->lds_z, ZArgs{0, 0, k.dev.smass}, c->tw, 0, c->stream,
               k.cfg.n);
  launch_ypass(+1, k.solo, 1, tx, c->lds_x, c->tw, 0, c->stream, k.cfg.n);
  launch_xpass(X_FWD, k.solo, 1, tx, c->lds_x, XArgs{0.f, 0.f, XF_OUT_SHAT}, c->tw, 0,
               c->stream, k.cfg.n);
  hmc_status st = check_launch(c);
  if (st != HMC_OK) return st;
  k.learned = true;
  k.dev.mass_flat = flat ? 1 : 0;
  return HMC_OK;
}

static hmc_status set_mass_kind(hmc_ctx* c, int32_t chain, const float* logvar_dev, bool flat) {
  if (!c || chain < -1 || chain >= (int)c->ch.size()) return fail(c, HMC_EINVAL, "bad argument");
  if (chain >= 0) {
    hmc_status st = set_mass_one(c, c->ch[chain], logvar_dev, flat);
    if (st != HMC_OK) return st;
  } else {
    for (auto& k : c->ch) {
      if (logvar_dev && k.cfg.n != c->ch[0].cfg.n)
        return fail(c, HMC_EINVAL, "chain -1 with a field needs chains of one grid size");
    }
    for (auto& k : c->ch) {
      hmc_status st = set_mass_one(c, k, logvar_dev, flat);
      if (st != HMC_OK) return st;
    }
  }
  // the mass tables follow the kind (and, for the diagonal variant, mean(v))
  hmc_status st = upload_desc(c);
  if (st != HMC_OK) return st;
  launch_tables(c->d_all, (int)c->ch.size(), c->stream);
  if ((st = check_launch(c)) != HMC_OK) return st;
  bool all = true, any = false;
  for (auto& kk : c->ch) {
    all &= kk.learned;
    any |= kk.learned;
  }
  c->learned = all;
  c->mass_mixed = any && !all;
  // captured graphs hold the old pass sequence
  for (auto& g : c->g_traj) (void)hipGraphExecDestroy(g.second);
  for (auto& g : c->g_sweep) (void)hipGraphExecDestroy(g.second);
  c->g_traj.clear();
  c->g_sweep.clear();
  return HMC_OK;
}

hmc_status hmc_set_mass(hmc_ctx* c, int32_t chain, const float* logvar_dev) {
  return set_mass_kind(c, chain, logvar_dev, false);
}

hmc_status hmc_set_mass_diagonal(hmc_ctx* c, int32_t chain, const float* logvar_dev) {
  return set_mass_kind(c, chain, logvar_dev, true);
}

}  // extern "C"

// Kernel declarations (definitions in kernels.hip).
#pragma once
#include "common.hpp"

namespace hmc {

// records a context-free failure for hmc_last_error(NULL) and returns st
int32_t record_free_error(int32_t st, const char* why);

// x-pass modes (k-space side of a leapfrog step; see kernels.hip)
enum XMode : int { X_INV = 0, X_FWD = 1, X_START = 2, X_STEP = 3, X_END = 4 };
// x-pass flags
enum XFlag : int {
  XF_SCALE = 1,     // X_INV / X_FWD: delta_hat is scaled per shell (joint move)
  XF_DOT = 2,       // X_FWD: accumulate per-shell Re(conj(delta_hat) g_hat)
  XF_OUT_ALT = 4,   // X_FWD: store g_hat into the backup buffer instead of grad_k
  XF_OUT_DK = 8,    // X_FWD: store into delta_k (forward transform of a real field)
  XF_NOSTORE = 16,  // X_FWD: do not store
  XF_OUT_SHAT = 32,  // X_FWD: store into the learned-mass transform F(D^(1/2))
  XF_PRIOR = 64,     // X_INV: scale delta_hat by sqrt(lambda_k) (prior draw)
};
// learned-mass passes
enum LMode : int { L_START = 0, L_DRIFT = 1, L_KICK = 2, L_KICK_LAST = 3 };
enum LZMode : int { LZ_FORCE = 0, LZ_VEL = 1 };
// z-pass modes (real-space side)
enum ZMode : int { Z_GRAD = 0, Z_NOISE = 1, Z_C2R = 2, Z_R2C = 3 };
enum ZFlag : int {
  ZF_WRITE_DR = 1,   // store delta to delta_r
  ZF_WRITE_DRN = 2,  // store delta to the proposal buffer
  ZF_DATA = 4,       // accumulate the data energy
  ZF_WARM = 8,       // Z_NOISE: Philox stream of the warm start instead of the momenta
};

struct XArgs {
  float kick;   // factor of eps for the kick
  float drift;  // factor of eps for the drift
  int flags;
};
struct ZArgs {
  int flags;
  uint32_t unused;
  const float* src;  // Z_R2C input (single-chain launches)
};

// LDS bytes a pass needs for size n (dynamic shared memory)
int xpass_lds_bytes(int n);
int zpass_lds_bytes(int n);
int xpass_tiles(int n);
int zpass_tiles(int n);
bool supported_n(int n);

// launches (grid = total tiles of the class, capped at `grid_cap` blocks)
// uniform_n: the N shared by every chain of the launch, or 0 for mixed sizes;
// plan: radix plan (0 .. kPlanCount - 1) of the single-size step pass (X_STEP),
// y passes and force pass (Z_GRAD) for N >= 64; other launches use plan 0
constexpr int kPlanCount = 4;
void launch_xpass(int mode, const ChainDev* ch, int nch, int total, int lds, XArgs a,
                  const float2* tw, int grid_cap, hipStream_t s, int uniform_n, int plan = 0);
void launch_ypass(int dir, const ChainDev* ch, int nch, int total, int lds, const float2* tw,
                  int grid_cap, hipStream_t s, int uniform_n, int buf = 0,
                  int plan = 0);  // buf: T, T2, T3
void launch_xpass_learned(int mode, const ChainDev* ch, int nch, int total, int lds, XArgs a,
                          const float2* tw, int grid_cap, hipStream_t s, int uniform_n);
void launch_zpass_learned(int mode, const ChainDev* ch, int nch, int total, int lds, ZArgs a,
                          const float2* tw, int grid_cap, hipStream_t s, int uniform_n);
void launch_mass_prep(int phase, const ChainDev* ch, int total_r, const float* logvar,
                      hipStream_t s);
// y-z plane pass (inverse y, C2R z, data force, R2C z, forward y in one kernel)
// for single-size launches of the grid sizes it supports
bool plane_pass_supported(int n);
void launch_yzpass(const ChainDev* ch, int nch, ZArgs a, const float2* tw, hipStream_t s, int n);
void launch_zpass(int mode, const ChainDev* ch, int nch, int total, int lds, ZArgs a,
                  const float2* tw, int grid_cap, hipStream_t s, int uniform_n, int plan = 0);
void launch_export(const ChainDev* ch, int nch, int sweep, double* rec, int32_t* acc,
                   hipStream_t s);
void launch_shell_lut(const ChainDev* ch, int n, hipStream_t s);
void launch_field_moments(const float* x, double* mean, double* m2, long long nv, long long count,
                          hipStream_t s);
void launch_warm_combine(const ChainDev* ch, int total_r, const float* mu, const float* logvar,
                         hipStream_t s);

// elementwise / reductions
void launch_coeff(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_alpha_sum(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_static_moments(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_obs_mask(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_moments(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_energy_k(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_energy_r(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_shell_dot(const ChainDev* ch, int nch, int total, hipStream_t s);
void launch_shell_power(const ChainDev* ch, int nch, int total, hipStream_t s,
                        int with_counts = 0);
void launch_shell_index(const ChainDev* ch, int total, int16_t* out, hipStream_t s);
void launch_commit(int what, const ChainDev* ch, int nch, int total_k, int total_r,
                   hipStream_t s);
void launch_copy_real(const ChainDev* ch, int total_r, const float* src, float* dst,
                      hipStream_t s);

// per-chain scalar kernels (one block per chain)
void launch_reduce_slot(const ChainDev* ch, int nch, int slot, int dst, int cls, hipStream_t s,
                        bool mean = false);
// column sums of tile partials; src 0 shpart / 1 mpart; mode: see kernels.hip
void launch_colsum(const ChainDev* ch, int nch, int width, int src, int cls, int dst, int mode,
                   hipStream_t s);
void launch_tables(const ChainDev* ch, int nch, hipStream_t s);
// the Philox draw index (trajectory or sweep) lives in device memory so that a
// captured graph can be replayed for any index
void launch_set_draw(uint32_t* p, uint32_t v, hipStream_t s);
void launch_accept(const ChainDev* ch, int nch, hipStream_t s);
void launch_draw_power(const ChainDev* ch, int nch, hipStream_t s);
void launch_draw_nbar_bias(const ChainDev* ch, int nch, hipStream_t s);
void launch_rj(int phase, const ChainDev* ch, int nch, int nb_max, hipStream_t s,
               int cls = kTileXY);

enum Commit : int { C_HMC = 0, C_RJ = 1 };
enum RjPhase : int { RJ_BEGIN = 0, RJ_STEP = 1, RJ_END = 2 };

}  // namespace hmc

// Per-chain device descriptor and layout constants shared by the kernels and
// the host runtime.  Every launch covers all chains of a context: block b
// finds its chain by the per-pass tile bases, then dispatches on N.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hmc {

constexpr int kThreads = 256;     // block size of the passes (a few elementwise kernels use 1024)
constexpr int kMaxBins = 128;
constexpr int kMaxSub = 32;
// doubles ahead of P_m in each chain's sweep record (dH, accepted, rj_dH,
// rj_accepted, status, rj_wall_hits)
constexpr int kRecHead = 6;
constexpr int kElemPerTile = 16384;  // elementwise kernels: elements per tile

// tile classes (index into ChainDev::tb)
enum TileClass : int { kTileXY = 0, kTileZ = 1, kTileR = 2, kTileK = 3, kTileClasses = 4 };

// per-tile float64 partial-sum slots (ChainDev::part[slot * maxtiles + tile])
enum PartSlot : int {
  kPartKin = 0, kPartPri = 1, kPartDat = 2, kPartAlpha = 3, kPartAux = 4, kPartSlots = 5
};

// float64 parameter block of one chain (ChainDev::P)
enum POff : int {
  // scalars
  kDcur = 0,     // data energy of the current state
  kK0 = 1, kPi0 = 2, kK1 = 3, kPi1 = 4, kD1 = 5,
  kDH = 6, kAcc = 7, kAbar = 8, kLogU = 9,
  kRjDH = 10, kRjAcc = 11, kRjU0 = 12, kRjK0 = 13, kStatus = 14, kDnew = 15,
  kRjStep = 16, kHK = 17, kHP = 18, kHD = 19, kGbar = 20, kLmean = 21,
  kRjHits = 22,  // joint move: reflections off the walls in the last move
  // arrays
  kLam = 32,                       // lambda_m (unitary), nb
  kSigma = kLam + kMaxBins,        // sigma_m, nb
  kTheta = kSigma + kMaxBins,      // joint move: theta, theta0, rho, mass, bounds, dU
  kTheta0 = kTheta + kMaxBins,
  kRho = kTheta0 + kMaxBins,
  kMth = kRho + kMaxBins,
  kLo = kMth + kMaxBins,
  kHi = kLo + kMaxBins,
  kDU = kHi + kMaxBins,
  kWall = kDU + kMaxBins,          // joint move: reflections per shell in the current move
  kNmodes = kWall + kMaxBins,
  kBias = kNmodes + kMaxBins,      // per subsample
  kNbar = kBias + kMaxSub,
  kS0 = kNbar + kMaxSub,
  kBsum = kS0 + kMaxSub,
  kNobs = kBsum + kMaxSub,
  kS1 = kNobs + kMaxSub,
  kS2 = kS1 + kMaxSub,
  kTsum = kS2 + kMaxSub,
  kPSize = kTsum + kMaxSub,
};

// float tables per shell (ChainDev::tf) and float64 tables (ChainDev::td)
enum TOff : int {
  kTInvLam = 0, kTInvMass = kMaxBins, kTSqrtMass = 2 * kMaxBins, kTScale = 3 * kMaxBins,
  kTSize = 4 * kMaxBins
};
enum TdOff : int { kDInvLam = 0, kDInvMass = kMaxBins, kDSize = 2 * kMaxBins };

struct ChainDev {
  int n, h, nb, nsub;
  long long nv, nh;  // N^3 and N*N*(N/2+1)
  float norm;        // N^(-3/2)
  float eps;
  uint64_t seed;
  uint32_t chain;
  uint32_t fixed_mask;
  double alpha_prior;
  double box;
  int tb[kTileClasses];   // first global tile of this chain per class
  int nt[kTileClasses];   // tiles of this chain per class
  int maxtiles;           // stride of the partial-sum slots
  int mass_flat;          // 1: real-space diagonal mass (k-space mass 1/mean(v) for every mode)
  // caller buffers
  const float* R;
  const float* counts;
  const float* growth;  // per-voxel growth factor D+, or null (D+ = 1)
  float2* dk;
  float2* pk;
  float2* gk;
  float* dr;
  float* alpha;
  float* beta;
  // workspace
  float2* T;
  float2* bdk;
  float2* bgk;
  float* drn;
  double* part;    // [kPartSlots][maxtiles]
  double* shpart;  // [nb][maxtiles]: per-shell partial sums of each tile
  double* mpart;   // [maxtiles][3 * nsub]
  // library-owned small device state
  double* P;       // parameter block (kPSize doubles)
  float* tf;       // float shell tables (kTSize)
  double* td;      // float64 shell tables (kDSize)
  const float* lmass;  // learned real-space mass factor sqrt(D_i), or null
  const uint32_t* draw;  // device counter: Philox draw index of the current trajectory/sweep
  // learned mass: two more intermediate grids, F(D^(1/2)) and D^(1/2) per voxel
  float2* T2;
  float2* T3;
  float2* shat;
  float* smass;
  signed char* lut;  // shell index of every q = |k|^2 in grid units (-1 at q = 0)
  // survey support: bit g of word w is set when one of the 4 voxels of group
  // 64 w + g (voxels 4 (64 w + g) .. + 3) has R^l > 0 for some subsample l
  unsigned long long* obs;
};

// Twiddle tables W_L^i = exp(-2 pi i i / L), float2, for every supported
// length; offsets in this order.
__host__ __device__ constexpr int tw_offset(int L) {
  return L == 4 ? 0 : L == 8 ? 4 : L == 16 ? 12 : L == 32 ? 28 : L == 64 ? 60
       : L == 96 ? 124 : L == 128 ? 220 : L == 192 ? 348 : L == 256 ? 540 : -1;
}
constexpr int kTwTotal = 796;

}  // namespace hmc

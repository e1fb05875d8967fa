// Device kernels of the GVM for gfx950 and their host-side launchers.
//
// Every launcher takes a *group* of requests of one kernel id and covers all
// of them with one persistent launch; a single request is a group of one, so
// a rank's result does not depend on what else runs with it (each output
// element is produced by the same code with the same operation order).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace gvm {

constexpr int kMaxGroup = 32;  // requests per grouped launch (kernel-argument capacity, < 2 KiB)

struct VecDesc {
  const float* a;
  const float* b;
  float* c;
  uint64_t n;
  uint64_t unit_begin;  // first work unit of this request in the group
};

struct VecGroup {
  uint32_t count;
  uint32_t pad;
  uint64_t total_units;
  VecDesc d[kMaxGroup];
};

struct BsDesc {
  const float* S;
  const float* K;
  const float* T;
  float* call;
  float* put;
  uint64_t n;
  uint64_t unit_begin;
};

struct BsGroup {
  uint32_t count;
  uint32_t pad;
  uint64_t total_units;
  float rate;
  float volatility;
  BsDesc d[kMaxGroup];
};

struct GemmDesc {
  const float* A;
  const float* B;
  float* C;
  uint32_t n;        // square size
  uint32_t tiles_n;  // tiles along the columns of C
  uint32_t unit_begin;
  uint32_t units;    // tiles of this request
};

constexpr int kGroupXcds = 8;  // MI355X: workgroup w is dispatched to XCD w % 8

struct GemmGroup {
  uint32_t count;
  uint32_t total_units;
  GemmDesc d[kMaxGroup];
  // Balanced launch (mixed sizes, one workgroup per tile): the units are cut
  // into 16 slices of equal k-step work, slice s = [cut[s], cut[s + 1]), and
  // each XCD takes two of them (csrc/gemm_balance.hpp): balanced = 1 two
  // neighbouring slices, balanced = 2 one from each end.  Filled by
  // finalize_gemm_group; set by the launcher.
  uint32_t cut[2 * kGroupXcds + 1];
  uint32_t balanced;
  uint32_t pad[2];
};

struct EpDesc {
  const uint64_t* key;   // (k0, k1)
  uint64_t* out;         // sx, sy (binary64 bit patterns), q[0..9]
  uint64_t* partial;     // one record of the same layout per work unit
  uint64_t n;            // pairs
  uint64_t unit_begin;
  uint64_t units;
};

struct EpGroup {
  uint32_t count;
  uint32_t pad;
  uint64_t total_units;
  EpDesc d[kMaxGroup];
};

// SGEMM tile configurations available to the tuner.  A configuration is a
// pure function of n (see gemm_config_for), so a request always runs with the
// same tiles whatever it is grouped with.
struct GemmConfig {
  int id;
  int bm, bn, bk;   // macro tile of one workgroup
  int wm, wn;       // waves along M and N (wave tile = bm/wm x bn/wn)
  bool bt;          // B staged k-contiguous in LDS (transposed), else row-major
};

int gemm_config_count();
const GemmConfig& gemm_config(int idx);
// Tile configuration used for size n (table written by the tuner, compiled in).
int gemm_config_for(uint64_t n);
// Override the table (tuner only): config index for every n, or -1 to restore.
void gemm_config_force(int idx);

constexpr uint64_t kVecUnit = 4096;   // elements per vector work unit
constexpr uint64_t kBsUnit = 4096;    // options per Black-Scholes work unit (the launcher
                                      // recounts the units for its launch shape)

// Persistent-grid launchers.  `grid_cap` bounds the number of workgroups
// (0 = default for the kernel).  Return hipSuccess or the launch error.
hipError_t launch_vecadd_group(const VecGroup& g, hipStream_t s, int grid_cap = 0);
hipError_t launch_vecmul_group(const VecGroup& g, hipStream_t s, int grid_cap = 0);
hipError_t launch_bs_group(const BsGroup& g, hipStream_t s, int grid_cap = 0);
// grid_cap >= total_units asks for one workgroup per tile; for a group of
// mixed sizes the tiles are then spread over the XCDs by their k-steps
// (GemmGroup.xcd_begin) instead of by count.
hipError_t launch_sgemm_group(const GemmGroup& g, int config_idx, hipStream_t s, int grid_cap = 0);
// EP-like tally: one launch over the work units of every request (partials),
// then one workgroup per request sums its partials.
hipError_t launch_ep_group(const EpGroup& g, hipStream_t s, int grid_cap = 0);

// Fill the unit bookkeeping of a group (unit_begin, tiles, totals).
void finalize_vec_group(VecGroup& g);
void finalize_bs_group(BsGroup& g);
void finalize_gemm_group(GemmGroup& g, int config_idx);
void finalize_ep_group(EpGroup& g);

}  // namespace gvm

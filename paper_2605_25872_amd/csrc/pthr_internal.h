// Internal interface between the C ABI (pthr_api.cpp) and the kernels
// (pthr_kernels.hip).  Not installed; the public interface is include/pthr.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace pthr {

// Counter word 0 of every Philox block: site | sweep << 16 | purpose << 24.
enum Purpose : uint32_t { kInit = 1, kMetro = 2, kAcu = 3, kHseed = 4, kPt = 5, kWalker = 6 };

// Local update of the PT clones (the reservoir clones use Metropolis with
// MicSA too).
enum Update : int { kMetropolis = 0, kHeatBath = 1, kMicsa = 2 };

enum Phase : uint32_t {
  kPhaseSweep = 1u,     // Metropolis sweeps of PT and/or ER clones
  kPhaseHoudayer = 2u,  // one Houdayer move per pair and T_k < t_acu
  kPhasePT = 4u,        // energies, PT chain, round trips, ER exchange
  kPhaseMeasure = 8u,   // observables into the obs buffer
  kPhaseLabels = 16u,   // canonical cluster labels into a caller buffer
  kPhaseClusterStats = 32u,  // sizes of the six largest clusters per overlap sign
};

// Problem geometry, identical for every sample of a context.
struct Geo {
  int L, V, Vh;      // lattice side, sites, sites per checkerboard colour
  int S;             // samples
  int NR, NT;        // replica groups, temperatures
  int NERG;          // reservoir clones per group
  int NPT, NER, C;   // PT clones (NR*NT), ER clones (NR*NERG), all clones
  int NW, NWPT;      // 32-clone spin words per site: all, PT only
  int K_acu;         // number of temperatures with T_k < t_acu (a prefix)
  int mode;          // 0 all-cluster, 1 single negative cluster
  int update;        // local update of the PT clones (Update)
  int micsa_refresh; // MicSA: PT sweeps between walker refreshes (>= 1)
  float exp_lo, exp_hi;  // FP64 Metropolis: factors of the float bounds on exp (set per launch:
                        // 1 -+ 2^-20, or 0 and +inf to take the FP64 polynomial for every test)
  uint32_t key0, key1;
};

// Device pointers into the caller's state buffer (layout in pthr_api.cpp).
struct State {
  uint32_t* t_dev;     // EMCS counter t (device-resident so captured graphs can be replayed)
  uint32_t* spins;     // [S][NW][V] words; bit b of word w at site index j is
                       // clone 32w+b (PT) or NPT+32(w-NWPT)+b (ER); j = colour*Vh + i/2
  void* J;             // [S][3][V] double (FP64) or float (FP32), natural site order
  int32_t* clone_at;   // [S][NR][NT]
  int32_t* er_head;    // [S][NR]
  uint8_t* pt_last;    // [S][NR][NT-1]
  uint32_t* pt_count;  // [S][NR][NT-1]
  double* pt_energy;   // [S][NPT] energies at the PT step (before the reservoir exchange)
  double* e_now;       // [S][NPT] energies of the configurations after the PT step and exchange
  uint8_t* rt_state;   // [S][NPT]
  uint64_t* rt_count;  // [S]
  uint32_t* status;    // [S]
  const double* beta64;  // [NT]
  const float* beta32;   // [NT] FP32 form's Metropolis factor (float)(beta log2 e)
  void* beta_clone;      // [S][C] Metropolis factor of every clone (FP64: beta; FP32: beta log2 e),
                         // kept by the PT kernel
  const double* T64;     // [NT] temperatures as given
  double* walker;        // [S][NPT] MicSA walker energy of every PT clone (FP32 form: float values)
  float* J_plane;        // [S][3][V] FP32 couplings in the spin words' plane order (j = colour*Vh + i/2),
                         // kept for the MicSA row kernel's scalar loads; null where that kernel
                         // does not take them
};

struct Obs {
  uint64_t* n_meas;
  double* acc;    // [S][NT][6]
  uint64_t* hist; // [NT][V+1]
};

struct Run {
  uint32_t phases;    // Phase bits
  int m_pt0, n_pt;    // PT sweep counter start and number of PT sweeps
  int m_er0, n_er;    // same for ER clones
  int do_reservoir;
  int sample_begin;   // first sample of this launch
  float early_beta;   // Metropolis tests of clones with beta >= early_beta use the exp early-out
  int32_t* labels;    // kPhaseLabels output [S][NR/2][K_acu][V]; kPhaseClusterStats output
                      // [S][NR/2][K_acu][2][kStatTop]
  int hou_moves;      // Houdayer moves labelled at once (set by the launcher)
  int hou_chunk;      // Houdayer moves whose flips are collected before they are applied (a
                      // multiple of hou_moves; set by the launcher)
  int meas_k;         // temperatures per pass of the row-parallel overlaps (0: per-site form)
  int e_current;      // measure: e_now holds the energies of the current configurations
  int clone_split;    // sweep: work-items per chunk of sites (set by the launcher)
  int sample_split;   // sweep: workgroups per sample, each taking every sample_split-th clone group
};

// Device status bits (per sample).
enum : uint32_t { kStatusUnionBound = 1u, kStatusFindBound = 2u };

struct Shape {
  int chunk;       // sites per work-item: 2, 4 or 8
  int threads;     // work-items per sample workgroup (multiple of 64, <= 1024)
  int split;       // sweep only: work-items sharing each chunk's clone words (1, 2 or 4)
  int parts;       // sweep only: workgroups sharing each sample's clone words (1, 2 or 4)
  int hou_occupancy;  // Houdayer only: the launch has more samples than CUs or shares the GPU
                      // with other work, so more workgroups per CU may pay over more moves at once
};

constexpr size_t kLdsMax = 160 * 1024;  // gfx950 LDS per workgroup
constexpr int kMaxHouMoves = 16;        // Houdayer moves labelled at once, at most
constexpr int kStatTop = 6;             // largest clusters reported per overlap sign

// Static device workspace of pthr_autotune_noalloc: room for one state
// buffer of up to this many bytes, on every device the library runs on.
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of that workspace on the current device.
hipError_t scratch_address(void** ptr);

size_t lds_bytes(const Geo& g, int fp_bytes);
// Houdayer moves labelled at once; lds_rows: the PT spin words in LDS, else
// rows read from global memory with the flips of C moves collected before
// they are applied (only with `occupancy`); M = 0 if one move does not fit.
struct HouPlan {
  int M, C;
  bool lds_rows;
};
HouPlan houdayer_plan(const Geo& g, int threads, bool stats, bool flips, bool occupancy);
int measure_rows_per_pass(const Geo& g, int threads, int fp_bytes);
// FP32 MicSA row kernel: reading the couplings through the scalar cache (from
// a plane-order copy in the state buffer) leaves LDS to the spin words; taken
// wherever LDS then holds two samples' spin words (the geometry: lattice side,
// PT spin words, permutation entries NR NT, PT clones).
bool micsa_scalar_couplings(int L, int NWPT, int n_cat, int NPT);
hipError_t launch_emcs(int precision, const Geo& g, const State& st, const Obs& ob, const Run& run,
                       const Shape& sh, int n_blocks, hipStream_t stream);
hipError_t launch_init(const Geo& g, const State& st, hipStream_t stream);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);
hipError_t launch_advance_t(const State& st, hipStream_t stream);
// Raises the dynamic-LDS limit of every kernel instantiation once per process.
hipError_t prepare_kernels(size_t lds_bytes);

}  // namespace pthr

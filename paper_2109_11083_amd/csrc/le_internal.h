// le_internal.h -- device-side layout shared by the host runtime and the
// kernels of the Lees-Edwards library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "le.h"

namespace le {

constexpr int kBlock = 256;        // threads per block of the streaming per-particle kernels
constexpr int kTile = 128;         // particles (= threads) per tile of the pair kernels
constexpr int kHalo = 2560;        // positions a tile stages in LDS (slot kHalo: far sentinel)
constexpr int kHaloSearch = 1536;  // the same for the list search alone (systems without a force-time halo)
static_assert(kHaloSearch <= kHalo, "the halo tables are sized for kHalo");
static_assert(kHalo % (4 * kTile) == 0, "halo staging loops assume whole rounds of the tile");
constexpr int kForceTPP = 4;       // threads per particle of the halo-layout force kernel
constexpr int kGlobalTPP = 1;      // threads per particle of the global-layout force kernel (2: one per sub-list)
static_assert(kHalo % (kForceTPP * kTile) == 0, "halo staging rounds of the force kernel");
constexpr int kMaxRows = 3;        // cell rows a tile may span and still be staged
constexpr int kPieces = 4;         // x-image pieces per (row, dy, dz) of a tile
constexpr int kPlainBatch = 8;     // padding of the plain list (LDS gathers in flight)
constexpr int kOtherBatch = 4;     // padding of the imaged / global lists
constexpr int kStressComps = 12;   // 6 kinetic + 6 virial partial sums per block
constexpr int kSlots = 64;         // words (one per 128-byte line) a block maximum is spread over
constexpr int kLineInts = 32;      // 32-bit words per 128-byte line
constexpr int kLineU64 = 16;       // 64-bit words per 128-byte line
constexpr int kSortParticles = 512;  // particles per block of the scan-and-permute pass (on average)
constexpr int kBinBlock = 2 * kBlock;  // particles per block of the binning pass (two per thread)

// Mutable per-simulation scalars that live on the device so that a step
// never needs the host: step counter, offset, rebuild bookkeeping.  Two
// copies alternate: the kernel that advances the step reads one and writes
// the other (every block reads, one block writes), so no block ever sees a
// half-updated state; the host passes the current copy to each launch.
struct alignas(64) Ctrl {
  int64_t step;          // index n of the current state
  int64_t rebuild_step;  // step of the last neighbour-list build (m)
  int64_t n_rebuilds;
  double Delta;          // offset of step n, in [0, L_x)
  double Delta_ref;      // offset at the last build
  double drift;          // sum over steps since the build of dt * max |peculiar velocity|
  int32_t pos_cur;       // which position buffer holds the current positions
  int32_t aux_cur;       // which velocity/force/tag buffer is current
  int32_t rebuild;       // 1: the lists are (being) rebuilt for this state
  int32_t wraps;         // whole L_x folds of the offset since the build
};

// Sticky status and telemetry shared by both control copies.
struct alignas(64) Flags {
  int32_t status;        // LE_OK or the first LE_E_* code latched by a kernel
  // largest neighbour count of the last build: max over kSlots words, one per
  // 128-byte line (block b updates word b mod kSlots)
  int32_t max_nb_slot[kSlots * kLineInts];
};

// Everything a kernel needs, passed by value.
struct Dev {
  // geometry and physics
  double Lx, Ly, Lz;
  double inv_lx, inv_ly, inv_lz;   // cells per unit length (n_a / L_a)
  double lx;                       // cell length along x
  double shear_rate, sv;           // gamma_dot and gamma_dot * L_y
  // velocity storage (LE_VEL_*): the peculiar velocity is c = u - c_sr (y - L_y/2) e_x,
  // the drift moves x by dt (u_x + drift_sr (y - L_y/2)), a face crossing jumps
  // u_x by -k_y jump_sv.  Lab storage: (gamma_dot, 0, gamma_dot L_y); peculiar
  // storage: (0, gamma_dot, 0).
  double c_sr, drift_sr, jump_sv;
  double dt, h;                    // time step and dt / (2 m)
  double gamma_m;                  // gamma * m
  double pref;                     // sqrt(24 gamma m kT / dt)
  double dpd_gamma, dpd_pref;      // DPD: gamma and sqrt(24 gamma kT / dt)
  double dpd_rc2, dpd_inv_rc;      // DPD: r_c^2 and 1 / r_c of the weight omega
  double mass;
  double eps24, sig2;              // 24 eps, sigma^2
  double rc2, rlist, rlist2;       // cutoff^2, list radius, list radius^2
  double fene_k, fene_r02;
  double angle_k;                  // cosine angle term of the chains (0: none)
  double force_cap;                // > 0: pair-force magnitude cap (warm-up of overlapping starts)
  double inv_vol;
  int32_t nx, ny, nz, ncell;
  int32_t n, np;                   // particles, padded stride (np > n: slot n is a far-away sentinel)
  int32_t K;                       // capacity of each of a particle's two sub-lists
  int32_t np2;                     // 2 * np: sub-list v = h * np + i of particle i, h = 0, 1
  int32_t chain_len;
  int32_t n_bonded;                 // n_chains * chain_len (tags >= n_bonded are free)
  int32_t precision;
  int32_t staged;                  // 1: partners in the tile's LDS halo; 0: all from global memory
  int32_t small_halo;              // 1: the list search stages at most kHaloSearch positions per tile
  // FP32 pre-test of the list build: r2 (float, tile-relative coordinates)
  // below nb_lo is certainly inside r_list^2, at or above nb_hi certainly
  // outside; in between the plain FP64 displacement decides.
  float nb_lo, nb_hi;
  uint32_t seed_lo, seed_hi;
  uint32_t dpd_key_hi;             // seed_hi ^ 0x44504421: key word of the DPD pair noise
  int32_t thermostat;              // LE_THERMO_*
  int32_t nblocks;                 // blocks of the pair kernels (= ntiles)
  // buffers (device)
  double* pos[2];                  // double4 [np] each (x, y, z, wrap counts along y and z)
  double* vel[2];                  // [3][np]
  double* frc[2];                  // [3][np] total force of the current step
  double* vt;                      // DPD only: double4 [np] (u_x, u_y, u_z, tag) of the current slots,
                                   // packed before each force evaluation (one gather per partner)
  int32_t* tag[2];                 // slot -> tag
  int32_t* slot_of_tag;            // tag -> slot
  int32_t bcap;                    // bucket capacity per cell
  int2* bucket;                    // [ncell][bcap] (tag, slot) of the particles binned into each
                                   // cell, in arrival order
  int32_t* cell_count;             // [ncell]
  int32_t* cell_start;             // [ncell + 1]
  // Neighbour lists: two sub-lists per particle (v = h * np + i, h = 0, 1,
  // alternate batches of 8 candidates of each stencil range).  Entry k of sub-list v lives in a
  // block of consecutive entries: blocks of 8 (one 16-byte load) for nl16, of
  // 4 for nlo; block b of sub-lists v, v+1, ... is contiguous.
  //   nl16  partners staged in the tile's LDS halo (any image): LDS index,
  //         element k at ((k/8)*np2 + v)*8 + k%8
  //   nlo   partners not staged: slot in global memory in the low kSlotBits
  //         bits, image code (pack_img) above them; element k at
  //         ((k/4)*np2 + v)*4 + k%4
  uint16_t* nl16;
  uint32_t* nlo;
  int32_t* n_plain;                // [np2] staged entries per sub-list, multiple of kPlainBatch
  int32_t* n_og;                   // [np2] global entries per sub-list, multiple of kOtherBatch
  int32_t* halo_slot;              // [ntiles][kHalo] slot staged at each LDS position
  uint8_t* halo_code;              // [ntiles][kHalo] image code of each staged position
  int32_t* tile_nstage;            // [ntiles] staged positions per tile
  int32_t ntiles;
  int32_t* bond;                   // [2][np] slot of the chain neighbour below/above, -1 if none
  double* partials;                // [nblocks][kStressComps] (nblocks = ntiles)
  double* obs_part;                // [ceil(n / kBlock)][3 * LE_MAX_BINS + 4] observable partials
  Ctrl* ctrl;                      // current control copy (see Ctrl)
  Ctrl* ctrl_other;                // the other control copy (written by a batched rebuild test)
  // running max of |c|^2 of the last drift (bits of doubles >= 0) in kSlots
  // words of kLineU64 stride; two arrays alternate with the control copies
  unsigned long long* vmax;
  unsigned long long* vmax_other;  // the speed-bound slots paired with ctrl_other
  unsigned long long* scan_status; // [sp_blocks] look-back words of the cell scan
  int32_t sp_cells, sp_blocks;     // cells per block of the scan-and-permute pass, and its blocks
  Flags* flags;
};

// Descriptor table of a batched launch: simulation k owns the blocks
// [start[k], start[k+1]) of the grid and reads its descriptor (a Dev kept in
// its own workspace, one per control copy) through dev[k].  Passed by value.
constexpr int kMaxBatch = 64;
struct Batch {
  int32_t nsims;
  int32_t start[kMaxBatch + 1];
  const Dev* dev[kMaxBatch];
};
struct BatchOut {
  double* ptr[kMaxBatch];  // per-simulation output (the stress sample of this step)
};

// Entries of the lists of global slots: slot | code << kSlotBits (codes use 7 bits).
constexpr int kSlotBits = 24;
constexpr uint32_t kSlotMask = (1u << kSlotBits) - 1u;
__host__ __device__ inline uint32_t og_entry(uint32_t slot, uint8_t code) {
  return slot | ((uint32_t)code << kSlotBits);
}

// Image code of an imaged neighbour: sx in [-3, 3], sy and sz in [-1, 1].
__host__ __device__ inline uint8_t pack_img(int sx, int sy, int sz) {
  return (uint8_t)((sx + 3) | ((sy + 1) << 3) | ((sz + 1) << 5));
}
__host__ __device__ inline void unpack_img(uint8_t c, int& sx, int& sy, int& sz) {
  sx = (int)(c & 7) - 3;
  sy = (int)((c >> 3) & 3) - 1;
  sz = (int)((c >> 5) & 3) - 1;
}

// Launchers (le_kernels.hip).  Each enqueues on `stream` and returns the
// hipError_t of the launch.
enum ForceMode { kForcesOnly = 0, kStepFused = 1, kStepLast = 2, kInitForce = 3, kDpdForce = 4 };

// launch_rebuild reads control copy d.ctrl and writes `next`, which the
// following launches must then be given.  control: advance the step first
// (after a drift); force: rebuild whatever the criterion says.
hipError_t launch_rebuild(const Dev& d, Ctrl* next, unsigned long long* next_vmax, hipStream_t s,
                          bool force, bool control);
hipError_t launch_kick_drift(const Dev& d, hipStream_t s);
// DPD steps: the force kernel (kDpdForce) only writes the total force; this
// kernel then applies the second half-kick (and, unless last, the next
// half-kick and drift), with kinetic stress partials when sample is set.
hipError_t launch_integrate(const Dev& d, hipStream_t s, bool last, bool sample);
hipError_t launch_force(const Dev& d, hipStream_t s, ForceMode mode, bool sample, double* f_out,
                        double* sample_out, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
hipError_t launch_stress_final(const Dev& d, hipStream_t s, double* out6, bool virial_only);
hipError_t launch_observables(const Dev& d, hipStream_t s, int nbins, double* out);
hipError_t launch_unwrapped(const Dev& d, hipStream_t s, double* out);
hipError_t launch_msd(const Dev& d, hipStream_t s, const double* ref, double* out2);
hipError_t launch_ctrl_copy(const Ctrl* src, Ctrl* dst, const unsigned long long* vsrc,
                            unsigned long long* vdst, hipStream_t s);
hipError_t launch_state_out(const Dev& d, hipStream_t s, double* x, double* u, int32_t* cell_of,
                            int32_t* order);
hipError_t launch_pairs_out(const Dev& d, hipStream_t s, int64_t* pairs, int64_t cap,
                            unsigned long long* counter);
hipError_t launch_load_state(const Dev& d, hipStream_t s, const double* x0, const double* u0,
                             const double* f0, int64_t step0, double Delta0);
hipError_t launch_status_out(const Dev& d, hipStream_t s, int32_t* out);

// Batched launchers: one launch over the blocks of every simulation of a
// batch (all of one kernel configuration, given by `cfg`, the host copy of any
// member's descriptor).  Batches by block kind: `par` one block per kBlock
// particles, `bin` one per kBinBlock particles, `scan` one per sp_cells cells,
// `tile` one per kTile particles,
// `one` one block per simulation; `cur` and `nxt` name the descriptors of the
// current and the other control copy.
hipError_t launch_store_dev(const Dev& a, const Dev& b, Dev* dst, hipStream_t s);
hipError_t launch_kick_drift_b(const Batch& par_cur, hipStream_t s);
hipError_t launch_rebuild_b(const Batch& bin_cur, const Batch& scan_nxt, const Batch& tile_nxt,
                            const Dev& cfg, hipStream_t s);
hipError_t launch_force_b(const Batch& tile_cur, const Batch& par_cur, const Dev& cfg, hipStream_t s,
                          ForceMode mode, bool sample);
hipError_t launch_integrate_b(const Batch& tile_cur, hipStream_t s, bool last, bool sample);
hipError_t launch_stress_final_b(const Batch& one_cur, const BatchOut& out, hipStream_t s);
hipError_t launch_offsets(double sr, double Lx, double Ly, double dt, int64_t step0, int64_t count,
                          double* out, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                         hipStream_t s);

// Offset of step n: fmod(gamma_dot L_y * (n dt), L_x) folded into [0, L_x).
// fmod is exact, so host and device agree bit for bit.
__host__ __device__ inline double le_offset(int64_t n, double dt, double sv, double Lx) {
  double t = (double)n * dt;
  double d = fmod(sv * t, Lx);
  if (d < 0.0) d += Lx;
  if (d >= Lx) d -= Lx;
  return d;
}

}  // namespace le

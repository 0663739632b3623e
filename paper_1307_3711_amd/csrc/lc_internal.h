// lc_internal.h -- device-side layout shared by the kernels and the host runtime of liblcmd.
//
// Every array lives in one caller-owned device allocation.  Particles of all clusters are
// concatenated: cluster c owns global slots [off_c, off_c + cap_c), off_c a multiple of 64 (a
// cluster's share is its capacity rounded up to 64, so every 64-slot group, the slots of one
// wave, belongs to a single cluster); inside a cluster, ions
// occupy local slots [0, n_ion) and electrons follow (initial ones, then spawned ones in
// ascending parent order).  Per-particle arrays are structure-of-arrays FP64 except the
// packed source records the Coulomb kernel reads (float4 or double4 {x, y, z, q}).
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdint>
#include <utility>

#include "../../include/lcmd.h"

namespace lc {

constexpr int kBlock = 256;          // threads per block of the particle-parallel kernels
constexpr int kGroup = 64;           // slots per group: clusters start on group boundaries
constexpr int kDiagQ = 48;           // doubles per per-block diagnostic partial
constexpr int kDiagBlocks = 64;      // at most this many blocks per cluster in the diagnostic reduction
constexpr int kDiagSlots = 512;      // slots per block of the diagnostic reduction (up to kDiagBlocks)
constexpr int kHist = 17;            // charge histogram bins 0..16

// Field partial components written per source split: Ex, Ey, Ez, phi.
constexpr int kComp = 4;

// Device error flags (latched, OR-ed).
constexpr int kFlagNonfinite = 1;
constexpr int kFlagCapacity = 2;

// Static per-cluster parameters (dimensionless), uploaded once by lc_create.
struct ClusterParams {
  int64_t off;          // first global slot
  int64_t cap;          // slots
  int64_t n_ion;        // ions in local slots [0, n_ion)
  int64_t n_steps;      // retire after this many steps (INT64_MAX: never)
  double weight;        // real particles per macroparticle
  double mass_ion;      // ion mass in m_e
  double kw;            // kappa * weight: source strength per unit charge number
  double a0;            // peak field
  double tau;           // Gaussian FWHM (1/w)
  double t_sin2;        // sin^2 envelope length (1/w)
  double delta;         // spawn offset (c/w); also the offset of the initial electrons
  double r0;            // cluster radius (c/w)
  double n_atoms;       // real atoms (Eq.(1))
  double field_au;      // atomic field units per a0
  double rate_scale;    // 1/w per atomic time unit
  // ADK constants per charge state Z (transition Z -> Z+1), in atomic units:
  //   log nu = adk_logc[Z] - adk_expo[Z] * log F - adk_f23[Z] / F,  valid if adk_ok[Z]
  double adk_logc[LC_MAX_Z];
  double adk_expo[LC_MAX_Z];
  double adk_f23[LC_MAX_Z];
  int32_t adk_ok[LC_MAX_Z];
  int32_t envelope;
  int32_t phase;
  int32_t z_max;
  int32_t ion_block0;   // first entry of this cluster in the ion-block table
  int32_t n_ion_blocks;
  int32_t polarization;  // LC_LINEAR_X or LC_CIRCULAR
  int64_t n3_off;
  double det_r2;        // squared detector distance (c/w)^2 (detectors on)
  double box;           // side of the periodic cube around the cluster (c/w); 0: open boundaries
  // collisional ionization (Lotz): outer-subshell electrons and binding energy (eV) per
  // charge state, a * 2 sqrt(2/(pi m_e)) (cm^3/s eV^(3/2)), the estimate's sphere, the
  // real electrons per cm^3 of one macro-electron in it, seconds per unit of time
  double lotz_q[LC_MAX_Z];
  double ci_ip_ev[LC_MAX_Z];
  double lotz_av;
  double ci_r2;
  double ne_per_macro;
  double s_per_unit;    // seconds per unit of time (1/w)
};

// Per-cluster dynamic state, written by the kernels.
struct ClusterDyn {
  int64_t n_cur;        // live particles
  int64_t n_base;       // particle count before this step's spawns
  int64_t dropped;      // spawns that found no free slot (cumulative)
  int64_t events;       // ionizations (cumulative)
  int64_t rec_count;    // diagnostic records written
  double ke_start;      // sum w M (gamma - 1) at t0 - dt/2
  double laser_e;       // E_x of the dipole field at t^n: a(t^n) sin(t^n)
  double laser_ey;      // E_y of the dipole field at t^n: -a(t^n) cos(t^n) if circular, else 0
  double env;           // a(t^n)
  int32_t tile0;        // first tile of this cluster in the step's tile enumeration
  int32_t n_tiles;      // tiles of this cluster this step
  int32_t i_blocks;     // target blocks this step
  int32_t active;       // 1 while step < n_steps
  double pairs;         // sum over the steps taken of n_cur^2 (pair interactions evaluated)
  double ci_nu[LC_MAX_Z];  // collisional rate n_e <sigma v> per charge state this step (1/w units)
  int64_t n_sched;      // particle count the current step's tiles were built for
  int64_t steps_done;   // steps this cluster has taken
};

// Run-wide constants passed by value to every kernel.
struct RunConst {
  double dt;
  double t0;
  double eps2;
  uint64_t seed;
  int32_t n_clusters;
  int32_t ionize;
  int32_t ofi_local;
  int32_t diag_every;
  int32_t max_records;
  int32_t n3_rows;      // M: partial rows per target block of the pair-once kernel (0: none)
  int64_t n_total;      // total slots (sum of capacities)
  double mec2_ev;       // electron rest energy (eV) for the absorbed-energy column
  int32_t det_on;       // ion detectors present
  int32_t boundary;     // LC_OPEN, LC_PERIODIC or LC_MIXED
  int32_t collisional;  // collisional ionization rate added to the tunnelling rate
  int32_t ci_blocks;    // blocks per cluster of the electron density/temperature reduction
  double cap_slot_mean; // sum of capacity^2 over sum of capacity: the capacity of a typical slot's cluster
  double det_cos2;      // cos^2 of the detectors' acceptance half-angle
  double t_switch;      // LC_MIXED: first time (1/w) with open boundaries
  int32_t max_ion_blocks;  // ion blocks (256 ions) of the largest cluster
  int32_t diag_blocks;     // diag_blocks_for() of the largest cluster: the diagnostic grid's width
};

// Blocks of the diagnostic reduction of a cluster with cap slots.  A function of the cluster's
// own capacity only, so a cluster's records do not depend on the rest of the ensemble.
__host__ __device__ inline int diag_blocks_for(int64_t cap) {
  const int64_t b = (cap + kDiagSlots - 1) / kDiagSlots;
  return (int)(b < 1 ? 1 : (b > kDiagBlocks ? kDiagBlocks : b));
}

// Periodic boundaries in force at time t (the step's t^n): always for LC_PERIODIC, before
// t_switch for LC_MIXED, never for LC_OPEN.  Host and device take the same decision.
__host__ __device__ inline bool periodic_at(const RunConst& rc, double t) {
  return rc.boundary == LC_PERIODIC || (rc.boundary == LC_MIXED && t < rc.t_switch);
}

// Pointers into the caller-owned state.
struct DevState {
  double* x;
  double* y;
  double* z;
  double* ux;
  double* uy;
  double* uz;
  double* wl;
  double* wc;
  double* wsp;
  double* kebar;
  float4* pos4;         // FP32 source records (LC_FP32_*)
  double4* posq;        // FP64 source records (LC_FP64)
  int8_t* Z;
  int32_t* gcl;         // cluster of each 64-slot group
  double* part;         // field partials [split][comp][slot]
  void* n3part;         // pair-once partial rows (float or double: the pair type), per cluster from cp.n3_off
  int32_t* flag;        // ionization flags [slot of ion]
  int32_t* ib_count;    // spawns per ion block
  int32_t* ib_off;      // exclusive prefix of ib_count over all ion blocks
  int32_t* ib_cluster;  // cluster of each ion block
  ClusterParams* cp;
  ClusterDyn* dyn;
  int32_t* order;       // clusters in descending capacity (tile order)
  int32_t* tile_start;  // [n_clusters + 1] first tile of each order position this step
  int32_t* tile_total;  // tiles this step
  int32_t* queue;       // persistent-kernel work counter
  int8_t* det_seen;     // 1 once an ion has been counted by the detectors [slot]
  unsigned long long* det_counts;  // [cluster][4][LC_DET_SLOTS] detected macro-ions
  double* det_edges;    // LC_DET_BINS + 1 energy bin edges (eV)
  int32_t* err;         // latched error flags
  int64_t* step;        // absolute index of the current step group's first step
  double* diag_part;    // [cluster][kDiagBlocks][kDiagQ]
  double* ci_part;      // [cluster][kDiagBlocks][2] electron count and kinetic energy in the sphere
  double* records;      // [cluster][max_records][LC_REC]
  double* laser_tab;    // [step - *laser_tab0][cluster][3]: a(t), E_x, E_y of the steps of a group
  int64_t* laser_tab0;  // step index of the table's first row
};

// Steps a laser table covers (runs whose schedule can be left out inside a group of steps).
constexpr int kLaserTabSteps = 256;
// Clusters up to which runs without ionization keep a laser table.
constexpr int kLaserTabClusters = 64;

struct ForceTiling {
  int R;
  int WJ;
  int T;
  int S;
  int persistent;
  int scalar_src;   // FP32: sources as SGPR operands (scalar loads) instead of LDS tiles
  int newton3;      // FP32 + FP64 accumulation: each unordered pair once on steps without phi
};

// How the field partials of a step are laid out for the kernels that read them: S FP64 split
// partials [split][comp][slot] (a pair-once pass leaves its field in split 0: S = 1).
struct FieldLayout {
  int S;
};


// Envelope a(t) of the laser field amplitude (Eq.(3) and the test envelopes).
__device__ inline double envelope(const ClusterParams& cp, double t) {
  switch (cp.envelope) {
    case LC_GAUSS_FIELD: {
      const double d = t - 2.0 * cp.tau;
      return cp.a0 * exp(-2.77 * d * d / (cp.tau * cp.tau));
    }
    case LC_GAUSS_INTENSITY: {
      const double d = t - 2.0 * cp.tau;
      return cp.a0 * exp(-1.385 * d * d / (cp.tau * cp.tau));
    }
    case LC_SIN2: {
      if (t <= 0.0 || t >= cp.t_sin2) return 0.0;
      const double s = sin(M_PI * t / cp.t_sin2);
      return cp.a0 * s * s;
    }
    default:
      return cp.a0;
  }
}

// Envelope and dipole laser field (E_x, E_y) of a cluster at time t (Eqs.(3)-(9), psi = t);
// the magnetic field follows as z^ x E.
__device__ inline void laser_values(const ClusterParams& cp, double t, double& env, double& ex, double& ey) {
  env = envelope(cp, t);
  ex = env * sin(t);
  ey = (cp.polarization == LC_CIRCULAR) ? -(env * cos(t)) : 0.0;
}

// Counters of one cluster as step n begins: with advance, the step just taken is counted
// (n_sched^2 pair interactions, if the cluster was active); then the active flag and the live
// count this step's field pass covers.
__device__ inline void begin_step_counts(const ClusterParams& cp, ClusterDyn& d, int advance, int64_t n) {
  if (advance && d.active) {
    d.pairs += (double)d.n_sched * (double)d.n_sched;
    d.steps_done += 1;
  }
  d.active = (n < cp.n_steps) ? 1 : 0;
  d.n_sched = d.n_cur;
}

// Bookkeeping of one cluster as step n (time t) begins: its counters and the laser value of
// step n.  The tile tables are the caller's business.
__device__ inline void begin_step_cluster(const ClusterParams& cp, ClusterDyn& d, int advance, int64_t n,
                                          double t) {
  begin_step_counts(cp, d, advance, n);
  double env, ex, ey;
  laser_values(cp, t, env, ex, ey);
  d.env = env;
  d.laser_e = ex;
  d.laser_ey = ey;
}

// Cluster of global slot g (one table entry per 64-slot group).
__device__ inline int slot_cluster(const DevState& s, int64_t g) { return s.gcl[g / kGroup]; }

// Cluster of the wave whose 64 slots start at group boundary g0 (wave-uniform: the index goes
// through readfirstlane, so the table and the cluster's parameters are read by scalar loads).
__device__ inline int wave_cluster(const DevState& s, int64_t g0) {
  return s.gcl[__builtin_amdgcn_readfirstlane((int)(g0 / kGroup))];
}

// Coulomb field of slot g from the partials of the last field pass, summed over the splits in
// split order (FP64).  g is a global slot, or a lane's offset in a group view (group_view).
template <typename I>
__device__ inline void field_sum(const DevState& s, const RunConst& rc, const FieldLayout& fl, I g, double& ex,
                                 double& ey, double& ez) {
  const int64_t n = rc.n_total;
  if (fl.S == 1) {  // one split (every pair-once step): plain loads, no loop
    ex = s.part[g];
    ey = (s.part + n)[g];
    ez = (s.part + 2 * n)[g];
    return;
  }
  ex = 0.0; ey = 0.0; ez = 0.0;
  for (int k = 0; k < fl.S; ++k) {
    const double* b = s.part + (int64_t)k * kComp * n;
    ex += b[g];
    ey += (b + n)[g];
    ez += (b + 2 * n)[g];
  }
}

// The state as seen from the 64-slot group that starts at slot g0 (wave-uniform): every
// per-slot array advanced to g0, so a lane reaches its slot by a 32-bit offset from a scalar
// base, one shared address register for all of them instead of a 64-bit address per array.
__device__ inline DevState group_view(const DevState& s, int64_t g0) {
  DevState v = s;
  v.x += g0; v.y += g0; v.z += g0;
  v.ux += g0; v.uy += g0; v.uz += g0;
  v.wl += g0; v.wc += g0; v.wsp += g0; v.kebar += g0;
  v.pos4 += g0; v.posq += g0;
  v.Z += g0; v.part += g0; v.det_seen += g0;
  return v;
}

// Pair-once rows (written by the pair-once Coulomb kernel, layout in force.hip): the partial
// sums of global slot g over the rows m = w, w + ways, w + 2 ways, ... < nb of its block, in
// that order (FP64).  Blocks of `ways` waves over 64 consecutive slots read them coalesced.
constexpr int kFoldWaves = 8;

// Waves per 64 slots of the fused fold and push.  A slot has one row per block of its cluster:
// with many rows (48 and up for a typical slot) 8 waves keep enough loads in flight (4 for FP64
// rows); with few, most of 8 waves would idle, so the count is the smallest of 2, 4, 8 that
// still launches about 4096 waves (4 per SIMD).  Measured: 20k-slot cluster (79 rows) 8 waves
// (FP32 rows; 4 waves 11.5 against 10.2 us); 256-cluster ensemble of 1.4M slots (about 33 rows)
// 2 waves, 8 % faster than 8.
inline bool fold_many_rows(const RunConst& rc, int B) { return rc.cap_slot_mean >= 48.0 * (double)B; }
inline int fold_waves(const RunConst& rc, int B, int precision) {
  if (fold_many_rows(rc, B)) return precision == LC_FP64 ? 4 : 8;
  const int64_t groups = (rc.n_total + 63) / 64;
  int fw = 2;
  while (fw < 8 && groups * fw < 4096) fw *= 2;
  return fw;
}

// The FP64 sum of slot g's pair-once rows m = w, w + ways, ... (the share of wave w of
// `ways`), in row order.  RPR > 0: rounds of RPR rows whose loads are all issued before the
// first add (the row bound is wave-uniform); RPR = 0: rounds of four rows, then single rows.
// Measured on the 20k cluster (79 rows, 8 waves per 64 slots, fold and push together): 1 row
// per round 11.1 us, 2 rows 10.2 us, 3 rows 10.4 us, RPR = 0 10.7 us, 5 rows 10.9 us, 10 rows
// 11.0 us (fewer loads in flight per wave are faster, down to two); 2 rows with 16 waves
// 12.4 us.  On the 256-cluster ensemble (2 waves per 64 slots, about 33 rows) RPR = 0 runs
// 0.15 % faster over the whole run than four-row rounds with the last one predicated.
template <typename Tr, int RPR = 0>
__device__ inline void n3_row_partial(const DevState& s, const RunConst& rc, int B, int64_t g, int c, int w,
                                      int ways, double& e0, double& e1, double& e2) {
  e0 = 0.0; e1 = 0.0; e2 = 0.0;
  const ClusterParams& cp = s.cp[c];
  const ClusterDyn& d = s.dyn[c];
  const int64_t l = g - cp.off;
  const int64_t K = l / B;
  const int64_t nb = (d.n_sched + B - 1) / B;
  const Tr* r = (const Tr*)s.n3part + cp.n3_off + (K * rc.n3_rows + w) * 3 * (int64_t)B + (l - K * B);
  const int64_t step = (int64_t)ways * 3 * B;
  if constexpr (RPR == 0) {
    // four-row rounds, then the rows left one at a time
    int64_t m = w;
    for (; m + 3 * ways < nb; m += 4 * ways, r += 4 * step) {
      const double a0 = (double)r[0], a1 = (double)r[B], a2 = (double)r[2 * B];
      const double b0 = (double)r[step], b1 = (double)r[step + B], b2 = (double)r[step + 2 * B];
      const double c0 = (double)r[2 * step], c1 = (double)r[2 * step + B], c2 = (double)r[2 * step + 2 * B];
      const double d0 = (double)r[3 * step], d1 = (double)r[3 * step + B], d2 = (double)r[3 * step + 2 * B];
      e0 += a0; e0 += b0; e0 += c0; e0 += d0;
      e1 += a1; e1 += b1; e1 += c1; e1 += d1;
      e2 += a2; e2 += b2; e2 += c2; e2 += d2;
    }
    for (; m < nb; m += ways, r += step) {
      e0 += (double)r[0];
      e1 += (double)r[B];
      e2 += (double)r[2 * B];
    }
  } else {
    for (int64_t m = w; m < nb; m += RPR * ways, r += RPR * step) {
      Tr a0[RPR], a1[RPR], a2[RPR];
#pragma unroll
      for (int i = 0; i < RPR; ++i) {
        if (m + (int64_t)i * ways < nb) {
          a0[i] = r[i * step];
          a1[i] = r[i * step + B];
          a2[i] = r[i * step + 2 * B];
        }
      }
#pragma unroll
      for (int i = 0; i < RPR; ++i) {
        if (m + (int64_t)i * ways < nb) {
          e0 += (double)a0[i];
          e1 += (double)a1[i];
          e2 += (double)a2[i];
        }
      }
    }
  }
}

// A kernel launch whose dispatch records start and end events when e0 is given (the kernel's
// own duration, without the gaps that events recorded separately on the stream add).
template <typename... P, typename... A>
inline void launch_timed(void (*kern)(P...), dim3 grid, dim3 block, size_t lds, hipStream_t st, hipEvent_t e0,
                         hipEvent_t e1, A&&... args) {
  if (e0) hipExtLaunchKernelGGL(kern, grid, block, (std::uint32_t)lds, st, e0, e1, 0u, std::forward<A>(args)...);
  else hipLaunchKernelGGL(kern, grid, block, lds, st, std::forward<A>(args)...);
}

// Host launchers (defined in force.hip / step.hip).
// A pass without the potential takes the pair-once kernel when ft.newton3 is set.
// fold_n3 = false leaves the rows unsummed for launch_fold_push.  begin_step (pair-once,
// non-persistent passes only): the launch also does the step bookkeeping of the schedule that
// was left out before it (the tile tables of the step before must still hold).  e0, e1: events
// the pair-once kernel's dispatch records at its start and end (timing; nullptr: none).
hipError_t launch_force(const DevState& s, const RunConst& rc, int precision, const ForceTiling& ft,
                        bool want_phi, bool pbc, int grid_blocks, hipStream_t st, bool fold_n3 = true,
                        bool begin_step = false, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// n3: build the pair-once tile tables (blocks of n3_block_size(ft)) instead of target blocks
// times splits.
hipError_t launch_schedule(const DevState& s, const RunConst& rc, const ForceTiling& ft, bool n3, bool advance,
                           hipStream_t st);
// Laser values of steps *step + 1 .. *step + steps - 1 of every cluster into the laser table
// (steps <= kLaserTabSteps), for force launches that take over the schedule's bookkeeping.
hipError_t launch_laser_table(const DevState& s, const RunConst& rc, int steps, hipStream_t st);
// e0, e1: events the push's dispatch records at its start and end (timing; nullptr: none).
hipError_t launch_push(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl, int64_t k,
                       bool diag, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// Push after a pair-once pass whose rows were not folded: the fold and the push in one kernel
// (the field is also left in split 0 for the ionization check).
hipError_t launch_fold_push(const DevState& s, const RunConst& rc, int precision, int B, int64_t k, bool diag,
                            hipStream_t st);
hipError_t launch_start_kick(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl,
                             hipStream_t st);
hipError_t launch_diag(const DevState& s, const RunConst& rc, const FieldLayout& fl, int64_t k, hipStream_t st);
hipError_t launch_ionize(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl, int64_t k,
                         int n_ion_blocks, hipStream_t st);
// Initial placement of cluster c on the device (Sec. II random atoms inside R0): n_ion ions,
// each with z_init electrons, and the cluster's live count n_ion (1 + z_init).
hipError_t launch_init_generate(const DevState& s, const RunConst& rc, int c, int64_t n_ion, int z_init,
                                hipStream_t st);
// Source records of every live slot for the field pass of a step (pbc: that step is periodic).
hipError_t launch_refresh_sources(const DevState& s, const RunConst& rc, int precision, bool pbc, hipStream_t st);

// Standalone field (lc_field).
hipError_t launch_field_standalone(int precision, int64_t n, const double* xyzq, double eps2, double* E,
                                   double* phi, void* work, const ForceTiling& ft, hipStream_t st);
size_t field_workspace_bytes(int precision, int64_t n, const ForceTiling& ft);
// Device address of the current device's lc_field_static workspace (LC_FIELD_STATIC_MAX_BYTES),
// looked up on the first call per device.
hipError_t field_scratch(void** out);

int force_tile_targets(const ForceTiling& ft);
int n3_block_size(const ForceTiling& ft);
ForceTiling regular_tiling(int precision, const ForceTiling& ft);
int n3_persistent_grid(int precision, const ForceTiling& ft, int64_t tiles, int cus);
int64_t n3_tiles(int64_t n, int B);
bool force_tiling_valid(int precision, const ForceTiling& ft);

}  // namespace lc

/*
 * lcmd.h -- C ABI of the MI355X laser-cluster molecular-dynamics library (liblcmd.so).
 *
 * Method: A. R. Holkundkar, "Parallel Implementation of 3D Molecular Dynamic Simulation
 * for Laser-Cluster Interaction" (arXiv:1307.3711), Sec. II.  One time step of a cluster
 * is: the Coulomb field on every macroparticle from every other charged macroparticle,
 * the laser field of Eqs.(4)-(9) under the Eq.(3) envelope in the dipole approximation, a
 * relativistic Boris push, and the Monte-Carlo optical-field-ionization check with the
 * ADK rate (P = 1 - exp(-nu dt) against a uniform draw 0 < alpha <= 1), which spawns an
 * electron next to each ionized atom.  Options of the same section: linear or circular
 * polarization, open, periodic or mixed boundaries of the simulation box, and the
 * collisional ionization rate added to the tunnelling rate; and the ion detectors of the
 * Sec. III anisotropy study.  Units are the paper's: fields in a0 = eE/(m_e w c) (b0 = a0),
 * time in 1/w, length in c/w, momentum u = gamma v / c, energy in m_e c^2.
 *
 * Conventions for every entry point:
 *   - Return value: LC_OK (0) or a negative lc_status.  No exceptions cross the ABI.
 *     lc_last_error() gives a text for the last failure on a handle.
 *   - Device memory is owned by the caller.  The library never allocates device memory:
 *     the caller queries lc_state_bytes(), allocates that many bytes (any allocator; 256-B
 *     alignment) and passes the pointer to lc_create(); lc_field() takes a caller-owned
 *     workspace sized by lc_field_workspace_bytes().  Host pointers stay owned by the
 *     caller and are only read or written during the call.
 *   - Work is enqueued asynchronously on the HIP stream given at creation (a hipStream_t
 *     passed as void*; NULL is the null stream).  Only lc_read_* and lc_autotune
 *     synchronize that stream.
 *   - Device-side failures (capacity overflow, non-finite state) are latched in device
 *     flags and reported by the next synchronizing call.
 *   - A handle is not thread-safe; use one handle per stream.
 */
#ifndef LCMD_H
#define LCMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LC_API_VERSION 6
#define LC_MAX_Z 16       /* size of the per-charge tables (charge states 0..15)        */
#define LC_REC 48         /* doubles per diagnostic record                              */
#define LC_DET_BINS 120   /* ion energy histogram: 20 log bins per decade, 1 eV .. 1 MeV */
#define LC_DET_SLOTS (LC_DET_BINS + 2) /* the bins plus underflow and overflow         */

typedef enum {
  LC_OK = 0,
  LC_E_INVALID = -1,      /* bad argument or configuration                               */
  LC_E_CAPACITY = -2,     /* a cluster ran out of slots for spawned electrons            */
  LC_E_NONFINITE = -3,    /* a position or momentum became NaN/Inf                       */
  LC_E_HIP = -4,          /* a HIP runtime call failed                                   */
  LC_E_STATE = -5,        /* call out of order (e.g. step before start)                  */
  LC_E_UNSUPPORTED = -6   /* valid request the library does not implement                */
} lc_status;

/* Pair arithmetic of the Coulomb direct sum. */
typedef enum {
  LC_FP64 = 0,            /* FP64 everywhere                                             */
  LC_FP32_ACC64 = 1,      /* FP32 pair terms, FP32 partial sums per source tile, FP64
                             accumulation across tiles; FP64 push and diagnostics         */
  LC_FP32_KAHAN = 2       /* as LC_FP32_ACC64 with Kahan-compensated FP32 partial sums    */
} lc_precision;

/* Envelope of the laser field amplitude a(t). */
typedef enum {
  LC_GAUSS_FIELD = 0,     /* Eq.(3) as printed: a0 exp[-2.77 (t - 2 tau)^2 / tau^2]       */
  LC_GAUSS_INTENSITY = 1, /* same with exponent 1.385 (tau is the intensity FWHM)         */
  LC_SIN2 = 2,            /* a0 sin^2(pi t / T), T = n_cycles * 2 pi, zero outside [0, T]  */
  LC_FLAT = 3             /* a0                                                          */
} lc_envelope;

typedef enum {
  LC_DIPOLE = 0,          /* field depends on time only (Sec. II dipole approximation)    */
  LC_PLANE_WAVE = 1       /* test mode: phase t - z, wave along +z; ionization must be off */
} lc_phase;

/* Boundaries of the simulation box (Sec. II): a cube of side box_r0 * R0 centred on each
 * cluster (the paper takes the inter-cluster distance R_IC = 20 R0).  Periodic: every pair
 * interacts through the nearest periodic copy of the partner (minimum image) and a particle
 * leaving the cube re-enters through the opposite face.  Mixed: periodic for the steps with
 * t^n < t_switch, open afterwards. */
typedef enum {
  LC_OPEN = 0,
  LC_PERIODIC = 1,
  LC_MIXED = 2
} lc_boundary;

/* Polarization of the laser field (Eqs.(4)-(9); the magnetic field is z^ x E in both). */
typedef enum {
  LC_LINEAR_X = 0,        /* E = a(t) (sin psi, 0, 0), B = a(t) (0, sin psi, 0)             */
  LC_CIRCULAR = 1         /* phi_E = 3 pi/2, phi_B = pi/2: E = a(t) (sin psi, -cos psi, 0),
                             B = a(t) (cos psi, sin psi, 0), every component at full a(t)  */
} lc_polarization;

typedef enum {
  LC_LASER_ONLY = 0,      /* ADK driven by the laser field strength (Sec. II)              */
  LC_LOCAL = 1            /* ADK driven by |E_Coulomb + E_laser| at the ion                */
} lc_ofi_field;

/* Run-wide settings. */
typedef struct {
  uint32_t struct_size;   /* sizeof(lc_config)                                          */
  int32_t precision;      /* lc_precision                                               */
  int32_t ionize;         /* 0: charges frozen; 1: ADK Monte-Carlo ionization each step */
  int32_t ofi_field;      /* lc_ofi_field                                               */
  double lambda_um;       /* laser wavelength (micrometres)                             */
  double dt;              /* time step in 1/w (> 0)                                      */
  double t0;              /* time of step 0 in 1/w                                       */
  double softening_nm;    /* Plummer softening length (> 0)                              */
  int32_t diag_every;     /* one diagnostic record every k steps (0: none)              */
  int32_t max_records;    /* records kept per cluster (ring buffer)                     */
  int32_t max_splits;     /* largest source split the tuner may use (1..64)             */
  int32_t max_pair_blocks;/* M >= 0: room for the pair-once kernel (lc_tuning.newton3) on  */
                          /*   clusters of up to M blocks; costs 12 M (LC_FP32_ACC64) or  */
                          /*   24 M (LC_FP64) bytes per slot, slots rounded up to 512 per */
                          /*   cluster plus 512 more (blocks of 192-384 slots do not      */
                          /*   divide 512); 0: not available; not for LC_FP32_KAHAN       */
  uint64_t seed;          /* Philox key word 0 (word 1 is the cluster index)            */
  double detector_r0;     /* ion detectors at this multiple of each cluster's R0 from   */
                          /*   its centre (Sec. III anisotropy study: 9); 0: none       */
  double detector_half_angle_deg; /* their acceptance half-angle, in (0, 90) (Sec. III: 30) */
  int32_t boundary;       /* lc_boundary; periodic and mixed need LC_FP64 or LC_FP32_ACC64 */
  int32_t collisional;    /* 1 (needs ionize = 1): add the collisional rate n_e <sigma v> to the
                             tunnelling rate (Sec. II nu_total = nu_ofi + nu_ci).  <sigma v> is the
                             Lotz electron-impact rate of the ion's outermost subshell averaged
                             over a Maxwellian, 2 sqrt(2/(pi m_e)) a q E1(P/T) / (P sqrt(T)) with
                             q = lotz_q[Z], P = ip_ev[Z], a = lotz_a; n_e and T = (2/3) <KE> come
                             from the electrons inside the sphere of radius R0 around the cluster
                             centre after each push, and apply to the ions inside it            */
  double box_r0;          /* side of the periodic cube in units of each cluster's R0 (> 0) */
  double t_switch;        /* LC_MIXED: first time (1/w) of open boundaries              */
} lc_config;

/* One cluster, in physical units.  Species data (Wigner-Seitz radius, mass, ionization
 * potentials) is input: the paper lists R_W for D, Ne, Ar and Xe after Eq.(1). */
typedef struct {
  double r0_nm;               /* cluster radius                                         */
  double rw_angstrom;         /* Wigner-Seitz radius: N_atoms = (R0/R_W)^3 (Eq.(1))      */
  double mass_u;              /* ion mass in atomic mass units                          */
  double ip_ev[LC_MAX_Z];     /* ionization potential of charge state k -> k+1 (eV)     */
  double intensity_wcm2;      /* peak intensity; a0 from Eq.(2)                          */
  int32_t envelope;           /* lc_envelope                                            */
  int32_t phase;              /* lc_phase                                               */
  double fwhm_fs;             /* tau of the Gaussian envelopes                          */
  double n_cycles;            /* length of the sin^2 envelope in laser periods          */
  int64_t n_ion;              /* ion macroparticles; they occupy slots [0, n_ion)       */
  int64_t capacity;           /* slots for ions + electrons (spawns included)           */
  double weight;              /* real particles per macroparticle; 0: N_atoms / n_ion   */
  int32_t z_max;              /* highest ion charge (<= LC_MAX_Z - 1)                    */
  int32_t polarization;       /* lc_polarization                                        */
  double electron_offset_nm;  /* distance of a spawned electron from its ion            */
  int64_t n_steps;            /* the cluster retires after this many steps (0: never)   */
  double lotz_q[LC_MAX_Z];    /* collisional ionization: electrons in the outermost     */
                              /*   subshell of charge state k (0: no collisional rate)  */
  double lotz_a;              /* Lotz constant a (cm^2 eV^2)                            */
} lc_cluster;

/* Tiling of the Coulomb kernel (the autotuner's search space).  Zeros mean "default". */
typedef struct {
  int32_t targets_per_lane;   /* R: 1, 2, 4 or 8 register-blocked targets per lane      */
  int32_t waves_per_target;   /* WJ: 1, 2 or 4 waves of a block share targets and split  */
                              /*     each LDS source tile, then reduce through LDS       */
  int32_t tile_sources;       /* T: sources staged in LDS per step (256..4096)          */
  int32_t j_splits;           /* S: source range split over S blocks (partials in HBM)  */
  int32_t persistent;         /* 1: persistent grid pulling tiles from a device queue   */
  int32_t scalar_sources;     /* FP32 modes: 1 reads source records through the scalar  */
                              /*   unit into SGPR operands instead of staging LDS tiles  */
  int32_t newton3;            /* LC_FP32_ACC64, LC_FP64: 1 evaluates each unordered pair  */
                              /*   once (in the handle's pair precision) and            */
                              /*   applies it to both particles (Newton's third law) on   */
                              /*   steps without a diagnostic record; (R, WJ) in {(1,1),  */
                              /*   (2,1), (1,2), (2,2), (4,2)}: blocks of B = (4/WJ) 64 R */
                              /*   slots, 256 threads; (R, R) for R = 3..6: blocks of     */
                              /*   B = 64 R slots, 64 R threads.  Needs ceil(capacity/B) */
                              /*   <= max_pair_blocks for every cluster.  Diagnostic     */
                              /*   steps (which need the potential) run the one-sided    */
                              /*   kernel with the other fields, and with R = 1 (FP32) or */
                              /*   2 (FP64), WJ = 4 when it has no such (R, WJ).          */
  int32_t reserved;
} lc_tuning;

typedef struct lc_sim lc_sim;

/* ---------------------------------------------------------------- simulation */

/* Host-side check of the pair-once partial rows (no device work).  The pair-once kernel cuts a
 * cluster into nb = ceil(capacity / B) blocks of B slots and writes, for target block K and
 * partner block m (both < nb), component d of local slot l at row element ((K M + m) 3 + d) B + l
 * of the cluster's share of 3 M (capacity rounded up to 512, plus 512) elements, M =
 * max_pair_blocks; the fold reads the same elements.  For the pair-once shape (R, WJ) (see
 * lc_tuning.newton3) out[0] = B, out[1] = nb, out[2] = the share in elements.  Returns LC_OK if
 * lc_set_tuning accepts this shape for a cluster of this capacity (its rows then stay inside
 * the share), LC_E_INVALID if it does not (nb > M, rows beyond the share) or the shape,
 * precision or sizes are invalid. */
int lc_pair_rows_fit(int32_t precision, int32_t R, int32_t WJ, int64_t capacity, int32_t max_pair_blocks,
                     int64_t out[3]);

/* Bytes of caller-owned device memory lc_create() needs; 0 if the arguments are invalid. */
size_t lc_state_bytes(const lc_config* cfg, const lc_cluster* clusters, int32_t n_clusters);

/* Create a handle over caller-owned device memory d_state (>= lc_state_bytes bytes) on
 * stream hip_stream.  Converts units on the host (Eq.(1), Eq.(2), kappa = r_e k, ADK
 * constants) and uploads the per-cluster tables.  LC_E_INVALID on a bad configuration
 * (non-positive dt or softening, z_max out of range, capacity < n_ion, periodic boundaries
 * with LC_FP32_KAHAN, collisional ionization without ionization, ...). */
int lc_create(lc_sim** out, const lc_config* cfg, const lc_cluster* clusters, int32_t n_clusters,
              void* d_state, size_t bytes, void* hip_stream);

/* Copy one cluster's initial macroparticles from host memory: n particles, positions
 * x_nm (n x 3, row-major, nanometres), momenta u (n x 3, gamma v / c), charge numbers Z
 * (ions >= 0 in slots [0, n_ion), electrons -1 after them).  LC_E_INVALID if n exceeds
 * the capacity or the ion/electron layout is violated. */
int lc_init_from_host(lc_sim* sim, int32_t cluster, int64_t n, const double* x_nm, const double* u,
                      const int8_t* Z);

/* Seeded initial placement on the device (Sec. II: the atoms of a cluster, Eq.(1) of them,
 * sit at random inside the sphere of radius R0 and are lumped into n_ion ion macroparticles
 * of weight N_atoms / n_ion; every ion starts with charge z_init and z_init electrons at
 * electron_offset_nm from it).  Draws from Philox4x64-10 keyed by (lc_config.seed, cluster
 * index): ion i takes the counter (i, 0, 0, 0), whose first three 64-bit words u1, u2, u3
 * (as ((w >> 11) + 1) 2^-53 in (0, 1]) place it at radius R0 u1^{1/3}, polar cosine 2 u2 - 1
 * and azimuth 2 pi u3; electron e = i z_init + k of ion i (0 <= k < z_init) takes (e, 0, 1, 0)
 * and its first two words give the polar cosine and azimuth of its offset.  Slots: the ions
 * in [0, n_ion), then the electrons grouped by parent; momenta zero.  cluster: one cluster
 * index, or -1 for every cluster.  LC_E_INVALID if z_init is outside [0, z_max] or
 * n_ion (1 + z_init) exceeds a capacity.  Synchronizes the stream; replaces lc_init_from_host
 * for the clusters it places. */
int lc_init_generate(lc_sim* sim, int32_t cluster, int32_t z_init);

/* Leap-frog start for every cluster: a field pass at t0, then the backward half kick
 * u^{-1/2} = u^0 - (Z/M)(dt/2)(E + v^0 x B).  Must follow lc_init_from_host or
 * lc_init_generate.  The paper does not say how the leap-frog is started; this backward half
 * kick with the full Lorentz force at t0 is the reading taken. */
int lc_start(lc_sim* sim);

/* Enqueue n_steps time steps: the field pass (minimum image on periodic steps), the push
 * (wrap into the periodic cube, detector check), diagnostics every diag_every steps, the
 * collisional estimate and the ionization check with spawns.  Asynchronous. */
int lc_step(lc_sim* sim, int64_t n_steps);

/* Capture steps_per_graph steps into one hipGraph that lc_step replays (0 turns graph
 * replay off).  Replays are used only where they line up with the diagnostic cadence.
 * No passage of the paper defines this call: its performance study (Sec. III, execution time
 * against cores and against macroparticle count, the N_part^2 law) counts whole time steps;
 * a step of a small cluster is a few short launches, and replaying many steps as one graph
 * removes the per-launch cost without changing any result (replays are bitwise identical to
 * direct launches).  In a run without ionization the captured pair-once steps also leave out
 * the per-step tile schedule (no particle count can change); the next field pass does its
 * bookkeeping, with the same results.  Returns LC_E_INVALID for a negative count. */
int lc_set_graph(lc_sim* sim, int32_t steps_per_graph);

/* Copy the latest max_records diagnostic records (LC_REC doubles each, in time order) of one
 * cluster to host memory; synchronizes the stream.  The records hold the observables the
 * paper reports as functions of time (Sec. III: average kinetic energy, as in the lumping
 * study of the deuterium cluster; the population of each ion charge state, as in the argon
 * charge-state fractions; absorbed energy) and the energy budget of the Sec. II model (laser
 * work on the particles, Coulomb potential energy).  records must hold max_records * LC_REC
 * doubles (caller-owned host memory); *n_out receives the number written.  Returns a latched
 * device error (LC_E_CAPACITY, LC_E_NONFINITE) if one occurred.  Record layout:
 *  0 t  1 step  2 N  3 N_ion  4 N_electron  5 KE(n+1/2)  6 KE(n)  7 PE(n)
 *  8 W_laser  9 W_coulomb  10 spawn KE  11-13 momentum  14-16 sum w Z E_C  17 sum w|Z||E_C|
 *  18 mean ion charge  19 absorbed eV per atom  20 dropped spawns  21 ionizations
 *  22 envelope a(t)  23 KE(-1/2) at start  24..40 macro-ion count per charge 0..16 */
int lc_read_diagnostics(lc_sim* sim, int32_t cluster, double* records, int32_t max_records,
                        int32_t* n_out);

/* Copy one cluster's state to host memory (any pointer may be NULL): positions x (n x 3,
 * units of c/w), momenta u (n x 3), Z (n), cumulative laser and Coulomb work per particle
 * wl, wc (n each).  cap bounds the rows written; *n_out receives the live count.
 * Synchronizes the stream. */
int lc_read_particles(lc_sim* sim, int32_t cluster, double* x, double* u, int8_t* Z, double* wl,
                      double* wc, int64_t cap, int64_t* n_out);

/* Coulomb field of one cluster's current positions (Sec. II force from every other charged
 * macroparticle of the cluster), from a field pass with the handle's tiling (the pair-once
 * kernel if the tiling selects it): E (n x 3 host doubles, field units a0), cap bounds the
 * rows written, *n_out receives the live count.  The pass overwrites the field partials of
 * the last step, which the next step recomputes before use; a cluster that has retired
 * (n_steps reached) is not part of the pass and its rows are not meaningful.  Synchronizes
 * the stream. */
int lc_read_field(lc_sim* sim, int32_t cluster, double* E, int64_t cap, int64_t* n_out);

/* Time-integrated ion energy distribution at the detectors of one cluster (the Sec. III
 * anisotropy study: detectors at distance D = detector_r0 * R0 from the cluster centre on
 * the x axis (laser polarization), the y axis and the z axis, both signs of each).  An ion
 * is counted once, at the end of the first step whose push takes it to a distance >= D,
 * with its kinetic energy M (gamma - 1) m_e c^2 (eV per real ion, momentum of that push);
 * every axis whose direction its position makes an angle below the half-angle with counts
 * it too.  counts (4 x LC_DET_SLOTS int64, host): row 0 every detected ion, rows 1..3 the
 * x, y and z axes; slot 0 holds energies below edges[0], slot k (1 <= k <= LC_DET_BINS)
 * energies in [edges[k-1], edges[k]), slot LC_DET_BINS + 1 energies >= edges[LC_DET_BINS].
 * Counts are macro-ions (multiply by the cluster weight for real ions) and are exact
 * integers, independent of scheduling.  edges_ev (LC_DET_BINS + 1 doubles, host) may be
 * NULL; edge k is 10^(k/20) eV.  LC_E_STATE if the handle has no detectors.  Synchronizes
 * the stream and returns a latched device error if one occurred. */
int lc_read_iedf(lc_sim* sim, int32_t cluster, int64_t* counts, double* edges_ev);

/* Current time-step index (host mirror of the device counter). */
int64_t lc_step_index(const lc_sim* sim);

/* Average device time (ms) of the push kernel (out_ms[0]) and of the ionization kernels
 * (out_ms[1], 0 when ionization is off) over reps back-to-back launches on the current state,
 * without field passes in between (the push reuses the last field).  Each push dispatch records
 * its own start and end; the ionization group (check, spawn) is bracketed by events on the
 * stream.  The state advances as if stepped.  A bandwidth probe of the particle-parallel
 * kernels; synchronizes the stream. */
int lc_time_particle_kernels(lc_sim* sim, int32_t reps, double out_ms[2]);

/* Work counters of one cluster: out[0] steps taken (a cluster stops at its n_steps),
 * out[1] live macroparticles, out[2] pair interactions evaluated (sum over its steps of
 * N^2, self pairs included), out[3] ionization events.  Synchronizes the stream. */
int lc_cluster_counters(lc_sim* sim, int32_t cluster, double out[4]);

/* Set or read the Coulomb kernel tiling used by this handle. */
int lc_set_tuning(lc_sim* sim, const lc_tuning* t);
int lc_get_tuning(const lc_sim* sim, lc_tuning* t);

/* Time candidate tilings of the Coulomb kernel on the handle's current state (restoring
 * it afterwards), keep the fastest one whose field matches the default tiling's to the
 * precision's tolerance, and append the result to cache_json (may be NULL).  Synchronizes
 * the stream. */
int lc_autotune(lc_sim* sim, const char* cache_json, lc_tuning* chosen);

/* Run n_steps steps directly (no graph) with HIP events recorded on the handle's stream
 * around each kernel group, and return per group the summed device time in ms and the
 * number of launches: index 0 the Coulomb kernel, 1 push, 2 diagnostics, 3 ionization.
 * With a pair-once tiling, group 0 holds the pair-once passes only: the one-sided pass of a
 * diagnostic step (which also computes the potential) is added to group 2, and the push
 * group includes the fold of the pair-once rows.  A pair-once dispatch records its events
 * itself (its own start and end); the other groups are bracketed by events on the stream.
 * Advances the simulation like lc_step.  Synchronizes the stream. */
int lc_profile_steps(lc_sim* sim, int64_t n_steps, double out_ms[4], int64_t out_launches[4]);

/* Write the whole device state and step index to a file / restore it into a handle
 * created with the same configuration.  Synchronize the stream. */
int lc_save_state(lc_sim* sim, const char* path);
int lc_load_state(lc_sim* sim, const char* path);

void lc_destroy(lc_sim* sim);

/* ---------------------------------------------------------------- the field alone */

/* Workspace bytes for lc_field with n particles, a precision and a tiling (NULL: default);
 * 0 for an invalid precision, tiling or n < 0.  One-sided tilings need S * 32 bytes per
 * particle plus the source records; a pair-once tiling (newton3 = 1, blocks of B slots) keeps
 * 3 n ceil(n / B) partial sums in the pair type, about 12 n^2 / B bytes in FP32 (47 GB at
 * n = 1M, B = 256) and twice that in FP64. */
size_t lc_field_workspace_bytes(int32_t precision, int64_t n, const lc_tuning* t);

/* Softened Coulomb field of n point sources on themselves (Sec. II force from every other
 * charged particle; Plummer softening eps):
 *   E_i = sum_{j != i} q_j (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^{3/2}
 *   phi_i = sum_{j != i} q_j / (|r_i - r_j|^2 + eps^2)^{1/2}        (if d_phi != NULL)
 * d_xyzq: device, 4 n doubles laid out x[n], y[n], z[n], q[n] (q in field units).
 * d_E: device, 3 n doubles out, laid out Ex[n], Ey[n], Ez[n].  d_work: caller-owned device
 * workspace of at least lc_field_workspace_bytes().  Asynchronous on hip_stream.
 * A tiling with newton3 = 1 computes E only (d_phi must be NULL).
 * LC_E_INVALID for n < 0, n > 2^30, eps2 <= 0, a workspace that is too small or not 256-byte
 * aligned, or an unknown tiling; LC_E_HIP when a launch fails (also for a request of more than
 * 2^31 - 1 tiles). */
int lc_field(int32_t precision, int64_t n, const double* d_xyzq, double eps2, double* d_E,
             double* d_phi, void* d_work, size_t work_bytes, const lc_tuning* t, void* hip_stream);

/* Allocation-free variant of lc_field for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results as lc_field (bitwise, for the same arguments and tiling), with the
 * workspace in a device array of LC_FIELD_STATIC_MAX_BYTES that the library holds on every
 * device it runs on until the process ends, instead of a caller-owned d_work.  The caller still
 * passes the inputs and outputs.  Calls nothing that allocates; the first call on a device
 * looks the array's address up (make it outside graph capture).  LC_E_INVALID as lc_field,
 * and when lc_field_workspace_bytes() for the request exceeds LC_FIELD_STATIC_MAX_BYTES.
 * Every call on a device shares that device's array: calls that overlap on one device (other
 * streams, other threads) race and give undefined results; calls on one stream are ordered. */
#define LC_FIELD_STATIC_MAX_BYTES (64u << 20)
int lc_field_static(int32_t precision, int64_t n, const double* d_xyzq, double eps2, double* d_E,
                    double* d_phi, const lc_tuning* t, void* hip_stream);

/* ---------------------------------------------------------------- surrogate network */
/* A small network 4-64-64-2 (SiLU hidden units) that maps standardized features of a
 * cluster run (log R0, log N_atoms from Eq.(1), log peak intensity, log pulse FWHM) to
 * standardized (log absorbed energy per atom, mean ion charge).  It is trained on ensemble
 * runs of the model above and answers in place of a run.  FP32 master weights and Adam
 * moments; BF16 weights, inputs, hidden activations and hidden-2 gradient in the products;
 * FP32 accumulation on the BF16 matrix cores.
 *
 * Parameter order (4,610 floats): W1 (64 x 4 row-major), b1 (64), W2 (64 x 64, W2[n][k] maps
 * hidden-1 unit k to hidden-2 unit n), b2 (64), W3 (2 x 64), b3 (2).
 * Device pointers below are caller-owned; d_state must hold lc_mlp_state_bytes() bytes
 * (256-B aligned).  Rows of d_X are 4 floats, rows of d_Y 2 floats. */
size_t lc_mlp_state_bytes(void);
int lc_mlp_n_params(void);

/* Upload FP32 master weights from host memory; zero the Adam moments and step count and
 * reset the scaler to identity.  Synchronizes the stream. */
int lc_mlp_set_params(void* d_state, const float* host_params, void* hip_stream);

/* Copy the master weights (4,610 floats) and the scaler (x mean[4], x std[4], y mean[2],
 * y std[2]) to host memory (either pointer may be NULL).  Synchronizes the stream. */
int lc_mlp_get_params(const void* d_state, float* host_params, float* host_scaler, void* hip_stream);

/* Population mean and standard deviation of every input and target column over n rows
 * (FP64 sums in row order), stored as the scaler.  Asynchronous. */
int lc_mlp_fit_scaler(void* d_state, const float* d_X, const float* d_Y, int64_t n, void* hip_stream);

/* steps Adam steps (lr, beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of `batch` rows
 * (32..256, a multiple of 32): step k uses rows d_rows[k*batch .. (k+1)*batch) of d_X/d_Y
 * (d_rows: steps*batch int32 in [0, n)).  Loss (1/(2B)) sum (y - t)^2 of each step goes to
 * d_loss[k] (may be NULL).  One workgroup runs all steps in a fixed order (bitwise
 * reproducible).  Asynchronous; an out-of-range row is replaced by row 0 and reported by
 * lc_mlp_status. */
int lc_mlp_train(void* d_state, const float* d_X, const float* d_Y, int64_t n, const int32_t* d_rows,
                 int32_t batch, int32_t steps, float lr, float* d_loss, void* hip_stream);

/* Gradient of the loss over one minibatch (rows d_rows[0..batch)) without updating the
 * weights: d_grad receives 4,610 floats in parameter order, d_loss one float. */
int lc_mlp_grad(void* d_state, const float* d_X, const float* d_Y, int64_t n, const int32_t* d_rows,
                int32_t batch, float* d_grad, float* d_loss, void* hip_stream);

/* Predict n rows: raw features in (standardized inside), de-standardized outputs out. */
int lc_mlp_infer(const void* d_state, const float* d_X, float* d_Y, int64_t n, void* hip_stream);

/* LC_E_INVALID if a training call met an out-of-range row, else LC_OK.  Synchronizes. */
int lc_mlp_status(const void* d_state, void* hip_stream);

/* ---------------------------------------------------------------- constants and errors */

/* Unit conversions the library uses (for cross-checks): out[0] kappa = r_e k,
 * out[1] atomic field units per a0, out[2] rate scale (1/w per atomic time unit),
 * out[3] a0 from Eq.(2) for intensity_wcm2, out[4] k in 1/nm, out[5] m_e c^2 in eV. */
int lc_units(double lambda_um, double intensity_wcm2, double out[6]);

const char* lc_error_string(int code);
const char* lc_last_error(const lc_sim* sim);
int lc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LCMD_H */

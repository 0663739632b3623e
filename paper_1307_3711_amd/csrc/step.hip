// step.hip -- particle-parallel kernels of one time step on gfx950: per-step schedule and
// laser value (S1), Boris push (S3), ionization check and electron spawning (S4),
// diagnostics (S5), the leap-frog start and the step counter.
//
// All of these are HBM- or latency-bound; they are plain 1-thread-per-particle kernels with
// coalesced FP64 structure-of-arrays access.  Reductions (diagnostics, spawn offsets) are
// done in a fixed order so every run is bitwise reproducible.
#include <algorithm>

#include "lc_internal.h"

namespace lc {

namespace {

// ----------------------------------------------------------------------------- helpers

__device__ inline double gm1(double ux, double uy, double uz) {
  // gamma - 1 = u^2 / (1 + gamma): no cancellation for slow heavy ions
  const double u2 = ux * ux + uy * uy + uz * uz;
  return u2 / (1.0 + sqrt(1.0 + u2));
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 64x64->128 multiplies per round,
// Weyl key schedule between rounds.
struct U64x4 {
  uint64_t v[4];
};

// 64 x 64 -> 128-bit product from four 32 x 32 -> 64-bit products with carries folded into
// their additions (each term stays below 2^64), both halves from the same partial products.
__device__ inline void mul64x64(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
  const uint32_t a0 = (uint32_t)a, a1 = (uint32_t)(a >> 32);
  const uint32_t b0 = (uint32_t)b, b1 = (uint32_t)(b >> 32);
  const uint64_t p00 = (uint64_t)a0 * b0;
  const uint64_t t = (uint64_t)a1 * b0 + (p00 >> 32);
  const uint64_t u = (uint64_t)a0 * b1 + (uint32_t)t;
  hi = (uint64_t)a1 * b1 + (t >> 32) + (u >> 32);
  lo = (u << 32) | (uint32_t)p00;
}

__device__ inline U64x4 philox(uint64_t k0, uint64_t k1, uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint64_t hi0, lo0, hi1, lo1;
    mul64x64(M0, c0, hi0, lo0);
    mul64x64(M1, c2, hi1, lo1);
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  U64x4 o;
  o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
  return o;
}

// Uniform draw in (0, 1] from the top 53 bits (the paper's 0 < alpha <= 1).
__device__ inline double unit_interval(uint64_t x) {
  return (double)((x >> 11) + 1ULL) * (1.0 / 9007199254740992.0);
}

constexpr uint64_t kPurposeIon = 0;
constexpr uint64_t kPurposeElectron = 1;
constexpr uint64_t kPurposeAlpha = 2;
constexpr uint64_t kPurposeDirection = 3;

// Coordinate x on the 32-bit grid of a periodic cube (is = 2^32 / L): the integer nearest
// x is, reduced modulo 2^32 (to [-2^31, 2^31] first, so the conversion is exact for any
// position), as the bit pattern of the FP32 record's component.
__device__ inline float grid_coord(double x, double is) {
  const double u = x * is;
  const double w = u - 4294967296.0 * floor(u * (1.0 / 4294967296.0) + 0.5);
  return __uint_as_float((uint32_t)(int64_t)rint(w));
}

// Source record of slot g for the field pass of a step: {x, y, z, q}; FP32 records of a
// periodic pass hold the grid coordinates and q (2^32 / L)^2 (the pair kernels' grid units).
template <typename I>
__device__ inline void write_source(const DevState& s, int precision, bool grid, double box, I g, double x,
                                    double y, double z, double q) {
  if (precision == LC_FP64) {
    s.posq[g] = make_double4(x, y, z, q);
  } else if (grid) {
    const double is = 4294967296.0 / box;
    s.pos4[g] = make_float4(grid_coord(x, is), grid_coord(y, is), grid_coord(z, is), (float)(q * (is * is)));
  } else {
    s.pos4[g] = make_float4((float)x, (float)y, (float)z, (float)q);
  }
}

// Laser electric field (ax, ay, 0) at time t and height z (Eqs.(4)-(9)); the magnetic field
// is z^ x E = (-ay, ax, 0) for both polarizations (b0 = a0).
// Periodic boundaries (Sec. II): a particle leaving the cube of side L centred on the cluster
// re-enters through the opposite face, x -> x - L floor(x / L + 1/2) in [-L/2, L/2).
__device__ inline double wrap_box(double x, double L) { return x - L * floor(x / L + 0.5); }

__device__ inline void laser_at(const ClusterParams& cp, const ClusterDyn& d, double t, double z, double& ax,
                                double& ay) {
  if (cp.phase == LC_DIPOLE) {
    ax = d.laser_e;
    ay = d.laser_ey;
  } else {
    ax = d.env * sin(t - z);
    ay = (cp.polarization == LC_CIRCULAR) ? -(d.env * cos(t - z)) : 0.0;
  }
}

// ----------------------------------------------------------------------------- schedule (S6)
// A single workgroup: per cluster, active flag, laser value at t^n, target blocks and tiles of
// step n; exclusive scan of tiles over clusters in `order` (largest first).  advance = 1 ends a step:
// it counts the step just taken (n_sched^2 pair interactions of every cluster that was
// active) and moves the device step index on; advance = 0 rebuilds the tables of the current
// step (after the tiling changed).  n3: tiles of the pair-once kernel, nb (nb + 1) / 2 per
// cluster for nb blocks of TI slots; otherwise target blocks of TI times S source splits.
// Step bookkeeping of the cluster at order position p for step n at time t; returns its tiles.
__device__ inline int32_t schedule_cluster(const DevState& s, int p, int TI, int S, int n3, int advance, int64_t n,
                                           double t) {
  const int c = s.order[p];
  const ClusterParams& cp = s.cp[c];
  ClusterDyn& d = s.dyn[c];
  begin_step_cluster(cp, d, advance, n, t);
  const int ib = d.active ? (int)((d.n_sched + TI - 1) / TI) : 0;
  const int32_t tiles = n3 ? (int32_t)((int64_t)ib * (ib + 1) / 2) : ib * S;
  d.i_blocks = ib;
  d.n_tiles = tiles;
  return tiles;
}

// Laser values of the steps n0 + 1 .. n0 + steps - 1 (n0: the current step index) of every
// cluster, with the schedule's arithmetic, for the force launches that take over the step
// bookkeeping inside a group of steps.  Row j holds step n0 + j (row 0 is not used).
__global__ __launch_bounds__(kBlock) void k_laser_table(DevState s, RunConst rc, int steps) {
  const int64_t n0 = *s.step;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i == 0) *s.laser_tab0 = n0;
  const int64_t j = i / rc.n_clusters;
  const int c = (int)(i - j * rc.n_clusters);
  if (j < 1 || j >= steps) return;
  const int64_t n = n0 + j;
  const double t = rc.t0 + (double)n * rc.dt;
  double env, ex, ey;
  laser_values(s.cp[c], t, env, ex, ey);
  double* row = s.laser_tab + 3 * (j * rc.n_clusters + c);
  row[0] = env;
  row[1] = ex;
  row[2] = ey;
}

// Up to 64 clusters: one wave, the scan across its lanes without barriers.
__global__ __launch_bounds__(64) void k_schedule_wave(DevState s, RunConst rc, int TI, int S, int n3, int advance) {
  const int p = threadIdx.x;
  const int64_t n = *s.step + advance;
  const double t = rc.t0 + (double)n * rc.dt;
  const int32_t tiles = (p < rc.n_clusters) ? schedule_cluster(s, p, TI, S, n3, advance, n, t) : 0;
  int32_t v = tiles;
  for (int o = 1; o < 64; o <<= 1) {  // inclusive scan over the lanes
    const int32_t u = __shfl_up(v, o, 64);
    if (p >= o) v += u;
  }
  if (p < rc.n_clusters) {
    s.tile_start[p] = v - tiles;
    s.dyn[s.order[p]].tile0 = v - tiles;
  }
  if (p == 63) {  // lanes past the last cluster add no tiles, so lane 63 holds the total
    s.tile_start[rc.n_clusters] = v;
    *s.tile_total = v;
    *s.queue = 0;
    if (advance) *s.step = n;  // every lane read the old index at the start
  }
}

__global__ __launch_bounds__(kBlock) void k_schedule(DevState s, RunConst rc, int TI, int S, int n3,
                                                     int advance) {
  constexpr int kWaves = kBlock / 64;
  __shared__ int32_t sh_wave[kWaves];
  __shared__ int32_t sh_carry;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int64_t n = *s.step + advance;
  const double t = rc.t0 + (double)n * rc.dt;
  if (tid == 0) sh_carry = 0;
  __syncthreads();
  for (int base = 0; base < rc.n_clusters; base += kBlock) {
    const int p = base + tid;
    const int32_t tiles = (p < rc.n_clusters) ? schedule_cluster(s, p, TI, S, n3, advance, n, t) : 0;
    int32_t v = tiles;
    for (int o = 1; o < 64; o <<= 1) {  // inclusive scan across the wave's lanes
      const int32_t u = __shfl_up(v, o, 64);
      if (lane >= o) v += u;
    }
    if (lane == 63) sh_wave[wv] = v;
    __syncthreads();
    int32_t off = sh_carry;  // tiles of earlier passes and earlier waves of this pass
    for (int q = 0; q < wv; ++q) off += sh_wave[q];
    if (p < rc.n_clusters) {
      const int32_t excl = off + v - tiles;
      s.tile_start[p] = excl;
      s.dyn[s.order[p]].tile0 = excl;
    }
    __syncthreads();  // every wave has read sh_carry and sh_wave
    if (tid == kBlock - 1) sh_carry = off + v;  // the last lane of the last wave: the pass total
    __syncthreads();
  }
  if (tid == 0) {
    s.tile_start[rc.n_clusters] = sh_carry;
    *s.tile_total = sh_carry;
    *s.queue = 0;
    if (advance) *s.step = n;  // every thread read the old index before the loop's barriers
  }
}

// ----------------------------------------------------------------------------- push (S3)
// Per-particle state the push reads (loaded by the caller, which can overlap it with the
// field's loads).
struct PState {
  double x, y, z, ux, uy, uz, wl, wc;
  int zc;
  int seen;  // detector flag (with detectors on)
};

template <typename I>
__device__ inline PState load_pstate(const DevState& s, const RunConst& rc, I g) {
  PState p;
  p.x = s.x[g]; p.y = s.y[g]; p.z = s.z[g];
  p.ux = s.ux[g]; p.uy = s.uy[g]; p.uz = s.uz[g];
  p.wl = s.wl[g]; p.wc = s.wc[g];
  p.zc = s.Z[g];
  p.seen = 1;  // the detector flag is loaded after the field (load_seen)
  return p;
}

// The detector flag of slot g, loaded after the particle state and the field: its test comes
// first in the push, and loads complete in order, so loading it last keeps every load of the
// push in flight at once.
template <typename I>
__device__ inline void load_seen(const DevState& s, const RunConst& rc, I g, PState& p) {
  if (rc.det_on) p.seen = s.det_seen[g];
}

// Ion detectors (Sec. III anisotropy study): an ion is counted once, when a push first takes it
// to the detector distance, in the energy slot of M (gamma - 1) m_e c^2 (eV per real ion) for
// every ion and for each axis whose direction its position is within the acceptance cone of.
// Counts are integers (order-independent atomics); the slot is the number of edges <= E.
// Called for ions not counted yet (the flag comes with the particle state).
template <typename I>
__device__ inline void detect_ion(const DevState& s, const RunConst& rc, const ClusterParams& cp, int c, I g,
                                  double x, double y, double z, double M, double ux, double uy, double uz) {
  const double r2 = x * x + y * y + z * z;
  if (r2 < cp.det_r2) return;
  s.det_seen[g] = 1;
  const double ev = M * gm1(ux, uy, uz) * rc.mec2_ev;
  int lo = 0, hi = LC_DET_BINS + 1;  // first edge index with edges[k] > ev, in [0, LC_DET_BINS + 1]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (s.det_edges[mid] <= ev) lo = mid + 1;
    else hi = mid;
  }
  unsigned long long* h = s.det_counts + (size_t)c * 4 * LC_DET_SLOTS + lo;
  atomicAdd(h, 1ull);
  const double cc[3] = {x, y, z};
  for (int a = 0; a < 3; ++a)
    if (cc[a] * cc[a] > rc.det_cos2 * r2) atomicAdd(h + (a + 1) * LC_DET_SLOTS, 1ull);
}

// Relativistic Boris step of live particle g (cluster c) at step index n in the Coulomb field
// (ecx, ecy, ecz) from state p: u^{n-1/2} -> u^{n+1/2}, x^n -> x^{n+1}, with the exact discrete work split
// W_L / W_C, optional KE(n) for the diagnostics, and the refresh of the source record the next
// field pass reads.  s is the view of the particle's 64-slot group and g its lane there.
template <int PREC>
__device__ inline void push_one(const DevState& s, const RunConst& rc, uint32_t g, int c, int64_t n, int diag,
                                double ecx, double ecy, double ecz, const PState& p) {
  const ClusterParams& cp = s.cp[c];
  const ClusterDyn& d = s.dyn[c];
  const double t = rc.t0 + (double)n * rc.dt;
  double x = p.x, y = p.y, z = p.z;
  double ax, ay;
  laser_at(cp, d, t, z, ax, ay);
  const int zc = p.zc;
  const double M = (zc < 0) ? 1.0 : cp.mass_ion;
  const double uox = p.ux, uoy = p.uy, uoz = p.uz;
  double unx = uox, uny = uoy, unz = uoz;
  const double go = sqrt(1.0 + uox * uox + uoy * uoy + uoz * uoz);
  if (zc != 0) {
    // E = E_C + E_L, E_L = (ax, ay, 0); B_L = (-ay, ax, 0)
    const double h = 0.5 * ((double)zc / M) * rc.dt;
    const double Ex = ecx + ax, Ey = ecy + ay, Ez = ecz;
    const double umx = uox + h * Ex, umy = uoy + h * Ey, umz = uoz + h * Ez;
    const double gm = sqrt(1.0 + umx * umx + umy * umy + umz * umz);
    const double tx = h * -ay / gm, ty = h * ax / gm, tz = h * 0.0 / gm;
    const double t2 = tx * tx + ty * ty + tz * tz;
    const double sx = 2.0 * tx / (1.0 + t2), sy = 2.0 * ty / (1.0 + t2), sz = 2.0 * tz / (1.0 + t2);
    const double upx = umx + (umy * tz - umz * ty);
    const double upy = umy + (umz * tx - umx * tz);
    const double upz = umz + (umx * ty - umy * tx);
    const double ux2 = umx + (upy * sz - upz * sy);
    const double uy2 = umy + (upz * sx - upx * sz);
    const double uz2 = umz + (upx * sy - upy * sx);
    unx = ux2 + h * Ex;
    uny = uy2 + h * Ey;
    unz = uz2 + h * Ez;
  }
  const double gn = sqrt(1.0 + unx * unx + uny * uny + unz * unz);
  if (zc != 0) {
    // M (gamma_new - gamma_old) = Z dt E.(u_old + u_new)/(gamma_old + gamma_new), linear in E
    const double cc = cp.weight * (double)zc * rc.dt / (go + gn);
    const double sx = uox + unx, sy = uoy + uny, sz = uoz + unz;
    s.wl[g] = p.wl + cc * (ax * sx + ay * sy + 0.0 * sz);
    s.wc[g] = p.wc + cc * (ecx * sx + ecy * sy + ecz * sz);
  }
  if (diag) s.kebar[g] = cp.weight * M * 0.5 * (gm1(uox, uoy, uoz) + gm1(unx, uny, unz));
  x += rc.dt * unx / gn;
  y += rc.dt * uny / gn;
  z += rc.dt * unz / gn;
  if (periodic_at(rc, t)) {
    x = wrap_box(x, cp.box);
    y = wrap_box(y, cp.box);
    z = wrap_box(z, cp.box);
  }
  s.ux[g] = unx; s.uy[g] = uny; s.uz[g] = unz;
  s.x[g] = x; s.y[g] = y; s.z[g] = z;
  // records for the field pass of step n + 1, in that step's form
  write_source(s, PREC, periodic_at(rc, rc.t0 + (double)(n + 1) * rc.dt), cp.box, g, x, y, z, cp.kw * (double)zc);
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(unx) && isfinite(uny) && isfinite(unz)))
    atomicOr(s.err, kFlagNonfinite);
  if (!p.seen && zc > 0) detect_ion(s, rc, cp, c, g, x, y, z, M, unx, uny, unz);  // only ion slots hold Z > 0
}

// One wave per 64-slot group: the group's cluster comes from the group table through scalar
// loads (its parameters and counters too), a retired cluster or a group past the live count
// leaves the whole wave at once, and the particle loads follow without a per-lane lookup.
// The slots are addressed through the group's view (scalar bases, 32-bit lane offsets): one
// address register instead of a 64-bit pair per array, 84 VGPRs (5 waves per SIMD).  Measured:
// held to 80 VGPRs (6 waves) it compiles without spills but runs 4 % slower, with fewer loads
// in flight per wave; at 72 (7 waves) it spills and runs 24 % slower.
// Two waves per workgroup: workgroups go out to the compute units in a fixed rotation, and
// with four waves a layout whose clusters alternate long live and long empty runs (capacity
// 8192, half live) put nearly all live workgroups on the same half of the units; measured on
// a pattern probe, two-wave groups keep every layout tried within 0.9 of the best case.
constexpr int kPushBlock = 128;

template <int PREC>
__global__ __launch_bounds__(kPushBlock) __attribute__((amdgpu_waves_per_eu(5)))
void k_push(DevState s, RunConst rc, FieldLayout fl, int64_t k, int diag) {
  const int64_t g0 = (int64_t)blockIdx.x * kPushBlock + kGroup * __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (g0 >= rc.n_total) return;
  const int c = wave_cluster(s, g0);
  const ClusterDyn& d = s.dyn[c];
  const uint32_t lane = threadIdx.x & 63;
  const int64_t l = g0 - s.cp[c].off + lane;
  if (!d.active || l >= d.n_cur) return;
  const DevState v = group_view(s, g0);
  // the particle state is loaded first so that its loads and those of the field are in flight
  // together (one memory round trip instead of two)
  PState ps = load_pstate(v, rc, lane);
  double ecx, ecy, ecz;
  field_sum(v, rc, fl, lane, ecx, ecy, ecz);
  load_seen(v, rc, lane, ps);
  push_one<PREC>(v, rc, lane, c, *s.step + k, diag, ecx, ecy, ecz, ps);
}

// Fold of the pair-once rows and push in one kernel: FW waves over one 64-slot group add
// their share of the rows, wave 0 combines them in order, keeps the field in split 0 (read by
// the ionization check) and pushes.  Wave 0 loads the particle state before its rows so both
// latencies overlap.  The group's cluster is uniform over the block (scalar loads).
template <int PREC, int FW, int RPR>
__global__ __launch_bounds__(64 * FW) void k_fold_push(DevState s, RunConst rc, int B, int64_t k, int diag) {
  __shared__ double red[FW - 1][3][64];
  const uint32_t lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g0 = (int64_t)blockIdx.x * kGroup;
  const int c = wave_cluster(s, g0);
  const ClusterDyn& d = s.dyn[c];
  const int64_t l0 = g0 - s.cp[c].off;
  if (!d.active || l0 >= d.n_cur) return;  // the whole block: retired cluster or empty group
  const DevState v = group_view(s, g0);
  const bool live = l0 + lane < d.n_cur;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  PState ps;
  if (live) {
    if (w == 0) ps = load_pstate(v, rc, lane);
    if (PREC == LC_FP64) n3_row_partial<double, RPR>(s, rc, B, g0 + lane, c, w, FW, e0, e1, e2);
    else n3_row_partial<float, RPR>(s, rc, B, g0 + lane, c, w, FW, e0, e1, e2);
  }
  if (w > 0) {
    red[w - 1][0][lane] = e0;
    red[w - 1][1][lane] = e1;
    red[w - 1][2][lane] = e2;
  }
  __syncthreads();
  if (w == 0 && live) {
    for (int q = 0; q < FW - 1; ++q) {
      e0 += red[q][0][lane];
      e1 += red[q][1][lane];
      e2 += red[q][2][lane];
    }
    v.part[lane] = e0;
    (v.part + rc.n_total)[lane] = e1;
    (v.part + 2 * rc.n_total)[lane] = e2;
    load_seen(v, rc, lane, ps);
    push_one<PREC>(v, rc, lane, c, *s.step + k, diag, e0, e1, e2, ps);
  }
}

// ----------------------------------------------------------------------------- start
// Backward half kick with the full Lorentz force at t0: u^{-1/2} = u^0 - (Z/M)(dt/2)(E + v x B);
// kebar receives w M (gamma^{-1/2} - 1) for the start energy.
__global__ __launch_bounds__(kBlock) void k_start_kick(DevState s, RunConst rc, FieldLayout fl) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= rc.n_total) return;
  const int c = slot_cluster(s, g);
  const ClusterParams& cp = s.cp[c];
  const ClusterDyn& d = s.dyn[c];
  if (g - cp.off >= d.n_cur) return;
  double ecx, ecy, ecz;
  field_sum(s, rc, fl, g, ecx, ecy, ecz);
  double ax, ay;
  laser_at(cp, d, rc.t0, s.z[g], ax, ay);
  const int zc = s.Z[g];
  const double M = (zc < 0) ? 1.0 : cp.mass_ion;
  double ux = s.ux[g], uy = s.uy[g], uz = s.uz[g];
  if (zc != 0) {
    const double h = 0.5 * ((double)zc / M) * rc.dt;
    const double gg = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    const double vx = ux / gg, vy = uy / gg, vz = uz / gg;
    // E_L = (ax, ay, 0), B = (-ay, ax, 0)
    const double fx = (ecx + ax) + (vy * 0.0 - vz * ax);
    const double fy = (ecy + ay) + (vz * -ay - vx * 0.0);
    const double fz = ecz + (vx * ax - vy * -ay);
    ux -= h * fx;
    uy -= h * fy;
    uz -= h * fz;
  }
  s.ux[g] = ux; s.uy[g] = uy; s.uz[g] = uz;
  s.kebar[g] = cp.weight * M * gm1(ux, uy, uz);
}

// Per-cluster sum of kebar in slot order (one block per cluster, fixed tree).
__global__ __launch_bounds__(kBlock) void k_sum_kestart(DevState s) {
  __shared__ double sh[kBlock];
  const int c = blockIdx.x;
  const ClusterParams& cp = s.cp[c];
  const int64_t ncur = s.dyn[c].n_cur;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < ncur; i += kBlock) acc += s.kebar[cp.off + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) s.dyn[c].ke_start = sh[0];
}

// ----------------------------------------------------------------------------- diagnostics (S5)
// Partial sums per (cluster, block), diag_blocks_for(capacity) blocks per cluster each taking
// every nb-th run of 256 slots; quantity layout:
//  0 KE(n+1/2)  1 KE(n)  2 PE  3 W_L  4 W_C  5 spawn KE  6-8 momentum  9-11 sum w Z E_C
//  12 sum w|Z||E_C|  13 ions  14 electrons  15 sum of ion charges  16..32 charge histogram
// Quantities 0-12 are FP64 sums per lane, added over the wave in a fixed order; 13-32 are
// integer tallies (wave ballots for the counts, a per-lane sum for the charges), exact in any order.
constexpr int kQ = 33;
constexpr int kQf = 13;  // floating-point quantities

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ inline int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__global__ __launch_bounds__(kBlock) void k_diag_partial(DevState s, RunConst rc, FieldLayout fl) {
  __shared__ double sh[4][kQ];
  const int c = blockIdx.y;
  const ClusterParams& cp = s.cp[c];
  const ClusterDyn& d = s.dyn[c];
  const int nb = diag_blocks_for(cp.cap);
  if (!d.active || (int)blockIdx.x >= nb) return;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double q[kQf];
#pragma unroll
  for (int i = 0; i < kQf; ++i) q[i] = 0.0;
  int zsum = 0;                            // this lane's sum of ion charges
  int n_ion = 0, n_el = 0, hist[kHist];    // the wave's counts (the same in every lane)
#pragma unroll
  for (int b = 0; b < kHist; ++b) hist[b] = 0;
  // every lane of a wave runs the same iterations, so every ballot sees the whole wave
  for (int64_t base = (int64_t)blockIdx.x * kBlock + kGroup * wv; base < d.n_cur; base += (int64_t)nb * kBlock) {
    const int64_t li = base + lane;
    const bool ok = li < d.n_cur;
    int zc = 0;
    if (ok) {
      const int64_t g = cp.off + li;
      zc = s.Z[g];
      const double M = (zc < 0) ? 1.0 : cp.mass_ion;
      const double w = cp.weight;
      const double ux = s.ux[g], uy = s.uy[g], uz = s.uz[g];
      double ex, ey, ez;
      field_sum(s, rc, fl, g, ex, ey, ez);
      double phi = 0.0;
      for (int k = 0; k < fl.S; ++k) phi += s.part[((int64_t)k * kComp + 3) * rc.n_total + g];
      q[0] += w * M * gm1(ux, uy, uz);
      q[1] += s.kebar[g];
      q[2] += 0.5 * w * (double)zc * phi;
      q[3] += s.wl[g];
      q[4] += s.wc[g];
      q[5] += s.wsp[g];
      q[6] += w * M * ux;
      q[7] += w * M * uy;
      q[8] += w * M * uz;
      q[9] += w * (double)zc * ex;
      q[10] += w * (double)zc * ey;
      q[11] += w * (double)zc * ez;
      q[12] += w * fabs((double)zc) * sqrt(ex * ex + ey * ey + ez * ez);
      if (zc >= 0) zsum += zc;
    }
    n_el += __popcll(__ballot(ok && zc < 0));
    n_ion += __popcll(__ballot(ok && zc >= 0));
#pragma unroll
    for (int b = 0; b < kHist; ++b) hist[b] += __popcll(__ballot(ok && zc == b));
  }
#pragma unroll
  for (int i = 0; i < kQf; ++i) {
    const double v = wave_sum(q[i]);
    if (lane == 0) sh[wv][i] = v;
  }
  zsum = wave_sum_int(zsum);
  if (lane == 0) {
    sh[wv][13] = (double)n_ion;
    sh[wv][14] = (double)n_el;
    sh[wv][15] = (double)zsum;
#pragma unroll
    for (int b = 0; b < kHist; ++b) sh[wv][16 + b] = (double)hist[b];
  }
  __syncthreads();
  if (threadIdx.x < kQ) {
    const int i = threadIdx.x;
    const double v = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
    s.diag_part[((int64_t)c * kDiagBlocks + blockIdx.x) * kDiagQ + i] = v;
  }
}

__global__ __launch_bounds__(64) void k_diag_final(DevState s, RunConst rc, int64_t k) {
  __shared__ double tot[kQ];
  const int c = blockIdx.x;
  const ClusterParams& cp = s.cp[c];
  ClusterDyn& d = s.dyn[c];
  if (!d.active) return;
  if (threadIdx.x < kQ) {
    double v = 0.0;
    const int nb = diag_blocks_for(cp.cap);
#pragma unroll 8
    for (int b = 0; b < nb; ++b) v += s.diag_part[((int64_t)c * kDiagBlocks + b) * kDiagQ + threadIdx.x];
    tot[threadIdx.x] = v;
  }
  __syncthreads();
  const int64_t slot = d.rec_count % rc.max_records;
  double* r = s.records + ((int64_t)c * rc.max_records + slot) * LC_REC;
  const int64_t n = *s.step + k;
  const int i = threadIdx.x;
  if (i < LC_REC) {
    double v = 0.0;
    if (i == 0) v = rc.t0 + (double)n * rc.dt;
    else if (i == 1) v = (double)n;
    else if (i == 2) v = (double)d.n_cur;
    else if (i == 3) v = tot[13];
    else if (i == 4) v = tot[14];
    else if (i >= 5 && i <= 10) v = tot[i - 5];
    else if (i >= 11 && i <= 16) v = tot[i - 5];
    else if (i == 17) v = tot[12];
    else if (i == 18) v = tot[13] > 0.0 ? tot[15] / tot[13] : 0.0;
    else if (i == 19) v = tot[3] * rc.mec2_ev / cp.n_atoms;
    else if (i == 20) v = (double)d.dropped;
    else if (i == 21) v = (double)d.events;
    else if (i == 22) v = d.env;
    else if (i == 23) v = d.ke_start;
    else if (i >= 24 && i < 24 + kHist) v = tot[16 + (i - 24)];
    r[i] = v;
  }
  __syncthreads();
  if (i == 0) d.rec_count += 1;
}

// ----------------------------------------------------------------------------- collisional rate
// Exponential integral E1(x) for x > 0: the power series -gamma - ln x - sum_k (-x)^k/(k k!)
// up to x = 1 (Abramowitz & Stegun 5.1.11), the continued fraction of A&S 5.1.22 (modified
// Lentz evaluation) beyond.
__device__ inline double expint_e1(double x) {
  if (x <= 1.0) {
    double t = 1.0, acc = 0.0;
    for (int k = 1; k < 100; ++k) {
      t = t * (-x / (double)k);
      const double add = t / (double)k;
      acc += add;
      if (fabs(add) <= 1e-18 * fabs(acc)) break;
    }
    return -0.57721566490153286061 - log(x) - acc;
  }
  double b = x + 1.0, cc = 1e300, dd = 1.0 / b, h = dd;
  for (int i = 1; i < 1000; ++i) {
    const double an = -(double)i * (double)i;
    b += 2.0;
    dd = 1.0 / (an * dd + b);
    cc = b + an / cc;
    const double del = cc * dd;
    h *= del;
    if (fabs(del - 1.0) <= 1e-16) break;
  }
  return h * exp(-x);
}

// Maxwellian Lotz rate coefficient (cm^3/s) of an ion with q outer electrons bound by P eV at
// electron temperature T eV; av = a 2 sqrt(2/(pi m_e)) in cm^3/s eV^(3/2).
__device__ inline double lotz_rate(double av, double q, double P, double T) {
  if (!(T > 0.0) || !(q > 0.0) || !(P > 0.0)) return 0.0;
  return av * q * expint_e1(P / T) / (P * sqrt(T));
}

// Electron count and kinetic energy (sum of gamma - 1) inside the sphere of radius R0 about
// the cluster centre: rc.ci_blocks blocks per cluster (sized by the largest capacity, at most
// kDiagBlocks) over its electron slots, fixed-order reductions (as the diagnostics).
__global__ __launch_bounds__(kBlock) void k_ci_partial(DevState s, RunConst rc) {
  __shared__ double sh[4][2];
  const int c = blockIdx.y;
  const ClusterParams& cp = s.cp[c];
  const ClusterDyn& d = s.dyn[c];
  double cnt = 0.0, ke = 0.0;
  if (d.active) {
    for (int64_t li = cp.n_ion + (int64_t)blockIdx.x * kBlock + threadIdx.x; li < d.n_cur;
         li += (int64_t)rc.ci_blocks * kBlock) {
      const int64_t g = cp.off + li;
      const double x = s.x[g], y = s.y[g], z = s.z[g];
      if (x * x + y * y + z * z < cp.ci_r2) {
        cnt += 1.0;
        ke += gm1(s.ux[g], s.uy[g], s.uz[g]);
      }
    }
  }
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const double a = wave_sum(cnt), b = wave_sum(ke);
  if (lane == 0) { sh[wv][0] = a; sh[wv][1] = b; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int i = threadIdx.x;
    s.ci_part[((int64_t)c * kDiagBlocks + blockIdx.x) * 2 + i] = ((sh[0][i] + sh[1][i]) + sh[2][i]) + sh[3][i];
  }
}

// n_e (cm^-3) and T = (2/3) <KE> (eV) from the partials in block order, then the rate of every
// charge state in units of 1/w.
__global__ __launch_bounds__(64) void k_ci_final(DevState s, RunConst rc) {
  __shared__ double sh_ne, sh_te;
  __shared__ double sh_part[kDiagBlocks][2];
  const int c = blockIdx.x;
  const ClusterParams& cp = s.cp[c];
  ClusterDyn& d = s.dyn[c];
  if (threadIdx.x < rc.ci_blocks) {  // the partials load in parallel, then add in block order
    sh_part[threadIdx.x][0] = s.ci_part[((int64_t)c * kDiagBlocks + threadIdx.x) * 2];
    sh_part[threadIdx.x][1] = s.ci_part[((int64_t)c * kDiagBlocks + threadIdx.x) * 2 + 1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double cnt = 0.0, ke = 0.0;
    for (int b = 0; b < rc.ci_blocks; ++b) {
      cnt += sh_part[b][0];
      ke += sh_part[b][1];
    }
    sh_ne = cnt * cp.ne_per_macro;
    sh_te = (cnt > 0.0) ? (2.0 / 3.0) * (ke / cnt) * rc.mec2_ev : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < LC_MAX_Z) {
    const int z = threadIdx.x;
    d.ci_nu[z] = sh_ne * lotz_rate(cp.lotz_av, cp.lotz_q[z], cp.ci_ip_ev[z], sh_te) * cp.s_per_unit;
  }
}

// ----------------------------------------------------------------------------- ionization (S4)
// ADK rate (1/w units) of charge state z at field strength fa (atomic units), zero below 1e-6.
__device__ inline double adk_nu(const ClusterParams& cp, int z, double fa) {
  if (!(fa >= 1e-6)) return 0.0;
  return exp(cp.adk_logc[z] - cp.adk_expo[z] * log(fa) - cp.adk_f23[z] / fa) * cp.rate_scale;
}

// Laser field strength |E_L(t^n)| of the cluster's step (the rate's field with LC_LASER_ONLY).
__device__ inline double laser_strength(const ClusterParams& cp, const ClusterDyn& d) {
  return (cp.polarization == LC_CIRCULAR) ? sqrt(d.laser_e * d.laser_e + d.laser_ey * d.laser_ey)
                                          : fabs(d.laser_e);
}

// Flag every ion whose uniform draw alpha in (0,1] falls below P = 1 - exp(-nu dt), nu the
// ADK rate at the driving field (plus the collisional rate inside the cluster sphere); count
// flags per ion block.  With the laser-only field the rate depends on the charge state alone,
// so the first 32 threads of a block evaluate P for every charge state (outside and inside the
// sphere) once, with the same arithmetic as the per-ion path of LC_LOCAL.  An ion whose P is
// exactly 0 cannot ionize (alpha > 0) and takes no draw.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_ionize_check(DevState s, RunConst rc, FieldLayout fl, int64_t k) {
  __shared__ double sh_p[2][LC_MAX_Z];
  const int ibk = blockIdx.x;
  const int c = s.ib_cluster[ibk];
  const ClusterParams& cp = s.cp[c];
  ClusterDyn& d = s.dyn[c];
  const int b = ibk - cp.ion_block0;
  const int64_t li = (int64_t)b * kBlock + threadIdx.x;
  if (b == 0 && threadIdx.x == 0) d.n_base = d.n_cur;
  const bool table = !rc.ofi_local;  // uniform over the launch
  if (table) {
    if (threadIdx.x < 2 * LC_MAX_Z) {
      const int z = threadIdx.x % LC_MAX_Z, inside = threadIdx.x / LC_MAX_Z;
      double P = 0.0;
      if (z < cp.z_max && cp.adk_ok[z]) {
        double nu = adk_nu(cp, z, laser_strength(cp, d) * cp.field_au);
        if (inside) nu += d.ci_nu[z];
        P = -expm1(-nu * rc.dt);
      }
      sh_p[inside][z] = P;
    }
    __syncthreads();
  }
  int flag = 0;
  if (d.active && li < cp.n_ion) {
    const int64_t g = cp.off + li;
    const int zc = s.Z[g];
    if (zc >= 0 && zc < cp.z_max && cp.adk_ok[zc]) {
      bool inside = false;
      if (rc.collisional) {
        const double x = s.x[g], y = s.y[g], z = s.z[g];
        inside = x * x + y * y + z * z < cp.ci_r2;
      }
      double P;
      if (table) {
        P = sh_p[inside ? 1 : 0][zc];
      } else {
        double ex, ey, ez;
        field_sum(s, rc, fl, g, ex, ey, ez);
        ex += d.laser_e;
        ey += d.laser_ey;
        double nu = adk_nu(cp, zc, sqrt(ex * ex + ey * ey + ez * ez) * cp.field_au);
        if (inside) nu += d.ci_nu[zc];
        P = -expm1(-nu * rc.dt);
      }
      if (P > 0.0) {
        const int64_t n = *s.step + k;
        const U64x4 r = philox(rc.seed, (uint64_t)c, (uint64_t)li, (uint64_t)n, kPurposeAlpha, 0);
        flag = (unit_interval(r.v[0]) < P) ? 1 : 0;
      }
    }
    s.flag[g] = flag;
  }
  const int cnt = __syncthreads_count(flag);
  if (threadIdx.x == 0) s.ib_count[ibk] = cnt;
}

// Exclusive prefix sum of the per-block flag counts over every ion block, in block order, in one
// workgroup: each pass covers 1024 x 16 blocks, thread t the run of 16 consecutive blocks at
// 16 t (its loads issued together), the run totals are scanned across the workgroup (lane
// shuffles within each wave, then across the 16 waves) with the carry of earlier passes, and
// each thread writes its run's offsets.  A cluster's ion blocks are contiguous, so the rank base
// of its block b is ib_off[ion_block0 + b] - ib_off[ion_block0].
constexpr int kScanRun = 16;
__global__ __launch_bounds__(1024) void k_ionize_scan(DevState s, int n_blocks) {
  __shared__ int32_t sh_w[16];
  __shared__ int32_t sh_carry;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) sh_carry = 0;
  for (int base = 0; base < n_blocks; base += 1024 * kScanRun) {
    const int i0 = base + tid * kScanRun;
    int32_t v[kScanRun];
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) v[k] = (i0 + k < n_blocks) ? s.ib_count[i0 + k] : 0;
    int32_t run = 0;
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) run += v[k];
    int32_t x = run;
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    __syncthreads();  // the previous pass's readers of sh_w and sh_carry are done
    if (lane == 63) sh_w[w] = x;
    __syncthreads();
    if (w == 0) {
      int32_t t = (lane < 16) ? sh_w[lane] : 0;
      for (int o = 1; o < 16; o <<= 1) {
        const int32_t y = __shfl_up(t, o, 64);
        if (lane >= o) t += y;
      }
      if (lane < 16) sh_w[lane] = t;
    }
    __syncthreads();
    const int32_t carry = sh_carry;
    int32_t off = carry + (w > 0 ? sh_w[w - 1] : 0) + x - run;
#pragma unroll
    for (int k = 0; k < kScanRun; ++k) {
      if (i0 + k < n_blocks) s.ib_off[i0 + k] = off;
      off += v[k];
    }
    __syncthreads();
    if (tid == 0) sh_carry = carry + sh_w[15];
  }
}

// Spawn one electron per flagged ion at slot n_base + (rank of the ion among this step's
// flagged ions, ascending ion index), next to the ion's new position with its momentum.
// The rank base of a block (flags of the cluster's earlier blocks) comes from the scan kernel
// when some cluster has more than kSpawnDirect ion blocks; otherwise every block adds up the
// counts of its cluster's earlier blocks itself, in parallel (integer sums: exact in any order),
// which saves the scan's launch and its latency.
constexpr int kSpawnDirect = 1024;
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_ionize_spawn(DevState s, RunConst rc, int64_t k, int scanned) {
  __shared__ int32_t sh_wave[4];
  __shared__ int32_t sh_pre[4];
  const int ibk = blockIdx.x;
  const int c = s.ib_cluster[ibk];
  const ClusterParams& cp = s.cp[c];
  ClusterDyn& d = s.dyn[c];
  const int b = ibk - cp.ion_block0;
  const int64_t li = (int64_t)b * kBlock + threadIdx.x;
  if (!d.active) return;
  int64_t base;
  if (scanned) {
    base = (int64_t)s.ib_off[ibk] - (int64_t)s.ib_off[cp.ion_block0];
  } else {
    int32_t pre = 0;
    for (int q = threadIdx.x; q < b; q += kBlock) pre += s.ib_count[cp.ion_block0 + q];
    for (int o = 32; o > 0; o >>= 1) pre += __shfl_xor(pre, o, 64);
    if ((threadIdx.x & 63) == 0) sh_pre[threadIdx.x >> 6] = pre;
    __syncthreads();
    base = (int64_t)sh_pre[0] + sh_pre[1] + sh_pre[2] + sh_pre[3];
  }
  const int flag = (li < cp.n_ion) ? s.flag[cp.off + li] : 0;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t ball = __ballot(flag);
  const int below = __popcll(ball & ((lane == 0) ? 0ULL : (~0ULL >> (64 - lane))));
  if (lane == 0) sh_wave[wv] = __popcll(ball);
  __syncthreads();
  int wave_off = 0;
  for (int q = 0; q < wv; ++q) wave_off += sh_wave[q];
  const int64_t n_base = d.n_base;
  const int64_t rank = base + wave_off + below;
  if (flag) {
    const int64_t e = n_base + rank;
    if (e < cp.cap) {
      const int64_t gi = cp.off + li;
      const int64_t ge = cp.off + e;
      const int64_t n = *s.step + k;
      const U64x4 r = philox(rc.seed, (uint64_t)c, (uint64_t)li, (uint64_t)n, kPurposeDirection, 0);
      const double ct = 2.0 * unit_interval(r.v[0]) - 1.0;
      const double ph = 2.0 * M_PI * unit_interval(r.v[1]);
      const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
      double xe = s.x[gi] + cp.delta * st * cos(ph);
      double ye = s.y[gi] + cp.delta * st * sin(ph);
      double ze = s.z[gi] + cp.delta * ct;
      if (periodic_at(rc, rc.t0 + (double)n * rc.dt)) {
        xe = wrap_box(xe, cp.box);
        ye = wrap_box(ye, cp.box);
        ze = wrap_box(ze, cp.box);
      }
      const double ux = s.ux[gi], uy = s.uy[gi], uz = s.uz[gi];
      s.x[ge] = xe; s.y[ge] = ye; s.z[ge] = ze;
      s.ux[ge] = ux; s.uy[ge] = uy; s.uz[ge] = uz;
      s.Z[ge] = -1;
      s.wl[ge] = 0.0;
      s.wc[ge] = 0.0;
      s.wsp[ge] = cp.weight * gm1(ux, uy, uz);
      const bool grid = periodic_at(rc, rc.t0 + (double)(n + 1) * rc.dt);  // records for step n + 1
      write_source(s, PREC, grid, cp.box, ge, xe, ye, ze, -cp.kw);
      const int znew = s.Z[gi] + 1;
      s.Z[gi] = (int8_t)znew;
      write_source(s, PREC, grid, cp.box, gi, s.x[gi], s.y[gi], s.z[gi], cp.kw * (double)znew);
    }
  }
  if (b == cp.n_ion_blocks - 1 && threadIdx.x == 0) {
    const int64_t total = base + sh_wave[0] + sh_wave[1] + sh_wave[2] + sh_wave[3];
    const int64_t room = cp.cap - n_base;
    const int64_t fit = total < room ? total : room;
    d.dropped += total - fit;
    d.events += fit;
    d.n_cur = n_base + fit;
    if (total > fit) atomicOr(s.err, kFlagCapacity);
  }
}

// ----------------------------------------------------------------------------- initial placement
// Sec. II: the atoms of a cluster sit at random inside the sphere of radius R0 and are lumped
// into ion macroparticles; each ion starts with charge z_init and z_init electrons at distance
// delta from it.  Draws: Philox4x64-10 keyed by (seed, cluster), counter (i, 0, 0, 0) for ion i
// (radius R0 u^{1/3}, polar cosine 2u - 1, azimuth 2 pi u), (e, 0, 1, 0) for electron
// e = i z_init + k of ion i (direction of its offset).  Slot order: ions, then electrons by
// parent.  One thread per slot; an electron's thread recomputes its parent's position.
__device__ inline void unit_direction(uint64_t wc, uint64_t wp, double& dx, double& dy, double& dz) {
  const double ct = 2.0 * unit_interval(wc) - 1.0;
  const double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  const double ph = 2.0 * M_PI * unit_interval(wp);
  dx = st * cos(ph);
  dy = st * sin(ph);
  dz = ct;
}

__device__ inline void ion_position(const RunConst& rc, int c, double r0, int64_t i, double& x, double& y,
                                    double& z) {
  const U64x4 r = philox(rc.seed, (uint64_t)c, (uint64_t)i, 0, kPurposeIon, 0);
  const double rad = r0 * cbrt(unit_interval(r.v[0]));
  double dx, dy, dz;
  unit_direction(r.v[1], r.v[2], dx, dy, dz);
  x = rad * dx;
  y = rad * dy;
  z = rad * dz;
}

__global__ __launch_bounds__(kBlock) void k_init_generate(DevState s, RunConst rc, int c, int64_t n_ion, int z_init) {
  const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t n0 = n_ion * (1 + (int64_t)z_init);
  const ClusterParams& cp = s.cp[c];
  if (l == 0) {
    s.dyn[c].n_cur = n0;
    s.dyn[c].n_base = n0;
  }
  if (l >= n0) return;
  const int64_t g = cp.off + l;
  double x, y, z;
  int zc;
  if (l < n_ion) {
    ion_position(rc, c, cp.r0, l, x, y, z);
    zc = z_init;
  } else {
    const int64_t e = l - n_ion;
    ion_position(rc, c, cp.r0, e / z_init, x, y, z);
    const U64x4 r = philox(rc.seed, (uint64_t)c, (uint64_t)e, 0, kPurposeElectron, 0);
    double dx, dy, dz;
    unit_direction(r.v[0], r.v[1], dx, dy, dz);
    x += cp.delta * dx;
    y += cp.delta * dy;
    z += cp.delta * dz;
    zc = -1;
  }
  s.x[g] = x; s.y[g] = y; s.z[g] = z;
  s.ux[g] = 0.0; s.uy[g] = 0.0; s.uz[g] = 0.0;
  s.Z[g] = (int8_t)zc;
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_refresh_sources(DevState s, RunConst rc, int grid) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= rc.n_total) return;
  const int c = slot_cluster(s, g);
  const ClusterParams& cp = s.cp[c];
  if (g - cp.off >= s.dyn[c].n_cur) return;
  write_source(s, PREC, grid != 0, cp.box, g, s.x[g], s.y[g], s.z[g], cp.kw * (double)s.Z[g]);
}

int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_schedule(const DevState& s, const RunConst& rc, const ForceTiling& ft, bool n3, bool advance,
                           hipStream_t st) {
  const int TI = n3 ? n3_block_size(ft) : force_tile_targets(ft);
  if (rc.n_clusters <= 64) k_schedule_wave<<<1, 64, 0, st>>>(s, rc, TI, ft.S, n3 ? 1 : 0, advance ? 1 : 0);
  else k_schedule<<<1, kBlock, 0, st>>>(s, rc, TI, ft.S, n3 ? 1 : 0, advance ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_laser_table(const DevState& s, const RunConst& rc, int steps, hipStream_t st) {
  if (!s.laser_tab || steps < 1 || steps > kLaserTabSteps || rc.n_clusters > kLaserTabClusters) return hipErrorInvalidValue;
  const int64_t n = (int64_t)steps * rc.n_clusters;
  k_laser_table<<<(int)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(s, rc, steps);
  return hipGetLastError();
}

hipError_t launch_push(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl, int64_t k,
                       bool diag, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const dim3 pb((unsigned)((rc.n_total + kPushBlock - 1) / kPushBlock));
  const int dg = diag ? 1 : 0;
  if (precision == LC_FP64) launch_timed(k_push<LC_FP64>, pb, dim3(kPushBlock), 0, st, e0, e1, s, rc, fl, k, dg);
  else launch_timed(k_push<LC_FP32_ACC64>, pb, dim3(kPushBlock), 0, st, e0, e1, s, rc, fl, k, dg);
  return hipGetLastError();
}

template <int PREC>
void fold_push_waves(int fw, int blocks, const DevState& s, const RunConst& rc, int B, int64_t k, int diag,
                     hipStream_t st) {
  // rounds of two rows where slots have many rows (fold_many_rows), else four-row rounds and
  // single rows
  if (fw <= 2) k_fold_push<PREC, 2, 0><<<blocks, 128, 0, st>>>(s, rc, B, k, diag);
  else if (fw <= 4 && fold_many_rows(rc, B)) k_fold_push<PREC, 4, 2><<<blocks, 256, 0, st>>>(s, rc, B, k, diag);
  else if (fw <= 4) k_fold_push<PREC, 4, 0><<<blocks, 256, 0, st>>>(s, rc, B, k, diag);
  else k_fold_push<PREC, 8, 2><<<blocks, 512, 0, st>>>(s, rc, B, k, diag);
}

hipError_t launch_fold_push(const DevState& s, const RunConst& rc, int precision, int B, int64_t k, bool diag,
                            hipStream_t st) {
  const int blocks = (int)((rc.n_total + 63) / 64);
  const int fw = fold_waves(rc, B, precision);
  if (precision == LC_FP64) fold_push_waves<LC_FP64>(fw, blocks, s, rc, B, k, diag ? 1 : 0, st);
  else fold_push_waves<LC_FP32_ACC64>(fw, blocks, s, rc, B, k, diag ? 1 : 0, st);
  return hipGetLastError();
}

hipError_t launch_start_kick(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl,
                             hipStream_t st) {
  (void)precision;
  k_start_kick<<<blocks_for(rc.n_total), kBlock, 0, st>>>(s, rc, fl);
  k_sum_kestart<<<rc.n_clusters, kBlock, 0, st>>>(s);
  return hipGetLastError();
}

hipError_t launch_diag(const DevState& s, const RunConst& rc, const FieldLayout& fl, int64_t k, hipStream_t st) {
  k_diag_partial<<<dim3(rc.diag_blocks, rc.n_clusters), kBlock, 0, st>>>(s, rc, fl);
  k_diag_final<<<rc.n_clusters, 64, 0, st>>>(s, rc, k);
  return hipGetLastError();
}

hipError_t launch_ionize(const DevState& s, const RunConst& rc, int precision, const FieldLayout& fl, int64_t k,
                         int n_ion_blocks, hipStream_t st) {
  if (n_ion_blocks <= 0) return hipSuccess;
  if (rc.collisional) {  // this step's electron density, temperature and collisional rates
    k_ci_partial<<<dim3(rc.ci_blocks, rc.n_clusters), kBlock, 0, st>>>(s, rc);
    k_ci_final<<<rc.n_clusters, 64, 0, st>>>(s, rc);
  }
  if (precision == LC_FP64) {
    k_ionize_check<LC_FP64><<<n_ion_blocks, kBlock, 0, st>>>(s, rc, fl, k);
  } else {
    k_ionize_check<LC_FP32_ACC64><<<n_ion_blocks, kBlock, 0, st>>>(s, rc, fl, k);
  }
  const int scanned = rc.max_ion_blocks > kSpawnDirect ? 1 : 0;
  if (scanned) k_ionize_scan<<<1, 1024, 0, st>>>(s, n_ion_blocks);
  if (precision == LC_FP64) k_ionize_spawn<LC_FP64><<<n_ion_blocks, kBlock, 0, st>>>(s, rc, k, scanned);
  else k_ionize_spawn<LC_FP32_ACC64><<<n_ion_blocks, kBlock, 0, st>>>(s, rc, k, scanned);
  return hipGetLastError();
}

hipError_t launch_init_generate(const DevState& s, const RunConst& rc, int c, int64_t n_ion, int z_init,
                                hipStream_t st) {
  const int64_t n0 = n_ion * (1 + (int64_t)z_init);
  k_init_generate<<<blocks_for(n0 > 0 ? n0 : 1), kBlock, 0, st>>>(s, rc, c, n_ion, z_init);
  return hipGetLastError();
}

hipError_t launch_refresh_sources(const DevState& s, const RunConst& rc, int precision, bool pbc, hipStream_t st) {
  if (precision == LC_FP64) k_refresh_sources<LC_FP64><<<blocks_for(rc.n_total), kBlock, 0, st>>>(s, rc, 0);
  else k_refresh_sources<LC_FP32_ACC64><<<blocks_for(rc.n_total), kBlock, 0, st>>>(s, rc, pbc ? 1 : 0);
  return hipGetLastError();
}

}  // namespace lc

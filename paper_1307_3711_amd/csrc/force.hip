// force.hip -- softened Coulomb direct sum on gfx950 (the paper's force calculation, Sec. II:
// every macroparticle feels every other charged macroparticle).
//
//   E_i   = sum_{j != i} q_j (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^{3/2}
//   phi_i = sum_{j != i} q_j / (|r_i - r_j|^2 + eps^2)^{1/2}        (diagnostic steps only)
//
// A direct sum is not a dense contraction, so this is VALU work, not MFMA.  Layout:
//   * a block of 256 threads (4 waves of 64) owns TI = (4/WJ) * 64 * R targets; each lane
//     keeps R targets in registers (register blocking over i);
//   * source records {x, y, z, q} are staged T at a time in LDS; every lane of a wave reads
//     the same LDS word at the same time (broadcast, no bank conflicts);
//   * WJ waves that share targets split each LDS tile between them and combine their sums
//     through LDS at the end, in a fixed order;
//   * the source range of a cluster is split over S blocks; each writes FP64 partial fields
//     part[s][comp][slot], which the push kernel adds in split order (deterministic);
//   * tiles of every cluster of an ensemble are enumerated in one launch: tile -> (cluster,
//     target block, split) through the per-step prefix table built by the schedule kernel;
//     the persistent variant pulls tiles from a device counter instead of blockIdx.
//
// Precision variants:
//   LC_FP64        : FP64 pair terms; 1/sqrt from v_rsq_f64 refined by the second-order
//                    series of (1 - e)^{-1/2} (one FMA-based residual, cubic convergence).
//   LC_FP32_ACC64  : FP32 pair terms with v_rsq_f32, FP32 sums within one LDS tile, FP64
//                    accumulation across tiles; tiles of equal-charge sources (the electron
//                    block, frozen or equal ion charges) use a loop with the charge factored out.
//   LC_FP32_KAHAN  : as above with Kahan-compensated FP32 sums within the tile.
#include <limits>
#include <mutex>

#include "lc_internal.h"

namespace lc {

namespace {

constexpr int kU = 8;  // inner-loop unroll; LDS tiles are padded to a multiple of it (times WJ)

struct TileMap {
  const int32_t* tile_start;   // [n_clusters + 1] prefix over clusters in `order`
  const int32_t* order;        // cluster at each order position
  const ClusterParams* cp;
  const ClusterDyn* dyn;
  const int32_t* tile_total;
  int32_t* queue;
  int n_clusters;
};

// Step bookkeeping a Coulomb launch takes over when no schedule launch precedes it (the tile
// tables of the step before still hold): the first wave of block 0 counts the step just taken
// and sets the next step's index and laser value (from the laser table, so that no
// transcendental function enters these kernels), fields no tile of the launch reads.
struct StepBegin {
  ClusterDyn* dyn;
  const ClusterParams* cp;
  int64_t* step;
  const double* tab;
  const int64_t* tab0;
  int n_clusters;
  int on;
};

// One wave: every lane loads the step index before lane 0 stores the next one.
__device__ inline void begin_step_wave(const StepBegin& b) {
  const int64_t n = *b.step + 1;
  const double* row = b.tab + 3 * (n - *b.tab0) * b.n_clusters;
  for (int c = threadIdx.x; c < b.n_clusters; c += 64) {
    ClusterDyn& d = b.dyn[c];
    begin_step_counts(b.cp[c], d, 1, n);
    d.env = row[3 * c];
    d.laser_e = row[3 * c + 1];
    d.laser_ey = row[3 * c + 2];
  }
  if (threadIdx.x == 0) *b.step = n;
}

template <typename Src>
struct ForceArgs {
  const Src* src;      // source/target records, global slot indexed
  double* part;        // [S][kComp][stride]
  int64_t stride;      // slots per partial component
  double eps2;
  int T;               // sources per LDS tile
  int S;               // splits
  int persistent;
  TileMap map;
  StepBegin begin;
};

__device__ inline void decode_tile(const TileMap& m, int t, int S, int& c, int& ib, int& s) {
  int lo = 0, hi = m.n_clusters - 1;
  while (lo < hi) {  // largest k with tile_start[k] <= t
    int mid = (lo + hi + 1) >> 1;
    if (m.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  c = m.order[lo];
  int local = t - m.tile_start[lo];
  ib = local / S;
  s = local - ib * S;
}

__device__ inline float rsq32(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/sqrt(x) to FP64 rounding: with y0 from v_rsq_f64 and e = 1 - x y0^2 (computed with an
// FMA), 1/sqrt(x) = y0 (1 - e)^{-1/2} = y0 (1 + e/2 + 3e^2/8 + O(e^3)); the hardware estimate
// leaves |e| below about 2^-22, so the truncated series is exact to far below an FP64 ulp.
__device__ inline double rsq64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  const double p = __builtin_fma(0.375, e, 0.5);
  return __builtin_fma(y * e, p, y);
}

// Minimum-image separation in a periodic cube of side L (iL = 1/L): the nearest periodic copy
// of the partner (Sec. II periodic boundaries); a separation inside (-L/2, L/2) is unchanged.
// FP64 records hold coordinates, and the copy is the rounded multiple of L.
__device__ inline double min_image(double d, double L, double iL) { return __builtin_fma(-L, __builtin_rint(d * iL), d); }

// FP32 records of a periodic pass hold the cube on a 32-bit grid (coordinate x as the integer
// nearest x 2^32 / L, modulo 2^32; the charge as q (2^32 / L)^2): the wrapping integer
// difference of two records is the minimum-image separation in grid units, one subtraction and
// one conversion per component, and the pair terms in grid units are the field in physical
// units (the potential is 2^32 / L times its physical value).
__device__ inline float grid_sep(float a, float b) {
  return (float)(int32_t)(__float_as_uint(a) - __float_as_uint(b));
}

template <typename T, bool PBC>
__device__ inline T pair_sep(T a, T b, T L, T iL) {
  if constexpr (!PBC) return a - b;
  else if constexpr (sizeof(T) == 4) return grid_sep(a, b);
  else return min_image(a - b, L, iL);
}

// eps^2 of a pass: in grid units, (eps 2^32 / L)^2, for FP32 records of a periodic pass.
template <typename T, bool PBC>
__device__ inline T pass_eps2(double eps2, double box) {
  if constexpr (PBC && sizeof(T) == 4) {
    const double is = 4294967296.0 / box;
    return (T)(eps2 * (is * is));
  } else {
    return (T)eps2;
  }
}

__device__ inline float n3_rsq(float x) { return rsq32(x); }
__device__ inline double n3_rsq(double x) { return rsq64(x); }

// ----------------------------------------------------------------------------- FP32 pair loop
// Sources [kb, kb + per) of the LDS tile against the lane's R targets.  UNIFORM: every source
// has the same charge q0 and the caller multiplies the sums by it (q r^-3 costs one multiply
// less per pair).  PHI: also the potential, with the self pair masked out by index.
// src is an LDS tile, or a global source array read with wave-uniform indices (the compiler
// then issues scalar loads and the pair arithmetic takes SGPR operands).  The sums and the
// Kahan compensations (cx..cpc) accumulate onto the caller's registers.
template <int R, bool PHI, bool KAHAN, bool UNIFORM, int U, bool PBC, typename P>
__device__ inline void pair_loop(P src, int kb, int per, int64_t jt, const int64_t* ii, const float* xi,
                                 const float* yi, const float* zi, float eps2f, float* fx, float* fy, float* fz,
                                 float* fp, float* cx, float* cy, float* cz, float* cpc) {
  for (int k = kb; k < kb + per; k += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4 sj = src[k + u];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float dx = pair_sep<float, PBC>(xi[r], sj.x, 0.f, 0.f);
        const float dy = pair_sep<float, PBC>(yi[r], sj.y, 0.f, 0.f);
        const float dz = pair_sep<float, PBC>(zi[r], sj.z, 0.f, 0.f);
        float r2 = __builtin_fmaf(dx, dx, eps2f);
        r2 = __builtin_fmaf(dy, dy, r2);
        r2 = __builtin_fmaf(dz, dz, r2);
        const float inv = rsq32(r2);
        float qinv = UNIFORM ? inv : sj.w * inv;
        const float sc = qinv * (inv * inv);
        if (KAHAN) {
          float y, tt;
          y = __builtin_fmaf(sc, dx, -cx[r]); tt = fx[r] + y; cx[r] = (tt - fx[r]) - y; fx[r] = tt;
          y = __builtin_fmaf(sc, dy, -cy[r]); tt = fy[r] + y; cy[r] = (tt - fy[r]) - y; fy[r] = tt;
          y = __builtin_fmaf(sc, dz, -cz[r]); tt = fz[r] + y; cz[r] = (tt - fz[r]) - y; fz[r] = tt;
        } else {
          fx[r] = __builtin_fmaf(sc, dx, fx[r]);
          fy[r] = __builtin_fmaf(sc, dy, fy[r]);
          fz[r] = __builtin_fmaf(sc, dz, fz[r]);
        }
        if (PHI) {
          if (jt + k + u == ii[r]) qinv = 0.f;  // exclude the self pair from the potential
          if (KAHAN) {
            float y = qinv - cpc[r]; float tt = fp[r] + y; cpc[r] = (tt - fp[r]) - y; fp[r] = tt;
          } else {
            fp[r] += qinv;
          }
        }
      }
    }
  }
}

// ----------------------------------------------------------------------------- FP32 body
template <int R, int WJ, bool PHI, bool KAHAN, bool SCALAR, bool PBC>
__device__ void tile_f32(const ForceArgs<float4>& a, const float4* __restrict__ gsrc, int t, float4* lds) {
  int c, ib, s;
  decode_tile(a.map, t, a.S, c, ib, s);
  const ClusterParams& cp = a.map.cp[c];
  const int64_t n = a.map.dyn[c].n_cur;
  const int64_t off = cp.off;
  constexpr int TG = 4 / WJ;
  constexpr int TI = TG * 64 * R;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;  // wave index, uniform
  const int g = w / WJ, jw = w % WJ;
  const int64_t i0 = (int64_t)ib * TI + (int64_t)g * 64 * R;

  const int64_t chunk = (n + a.S - 1) / a.S;
  const int64_t j0 = (int64_t)s * chunk;
  const int64_t j1 = (j0 + chunk < n) ? (j0 + chunk) : n;

  float xi[R], yi[R], zi[R];
  int64_t ii[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ii[r] = i0 + r * 64 + lane;
    float4 p = (ii[r] < n) ? a.src[off + ii[r]] : make_float4(0.f, 0.f, 0.f, 0.f);
    xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
  }
  double ex[R], ey[R], ez[R], ep[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { ex[r] = ey[r] = ez[r] = ep[r] = 0.0; }
  const float eps2f = pass_eps2<float, PBC>(a.eps2, cp.box);

  if constexpr (SCALAR) {
    // Sources straight from global memory with wave-uniform indices: scalar loads, SGPR
    // operands, no LDS traffic and no block barriers in the loop.  The WJ waves sharing these
    // targets take consecutive sub-ranges of the split; each wave walks its sub-range in
    // segments of T sources, with a per-segment uniform-charge check (wave vote).
    const int64_t sub = (j1 - j0 + WJ - 1) / WJ;
    const int64_t w0 = j0 + (int64_t)jw * sub;
    const int64_t w1 = (w0 + sub < j1) ? (w0 + sub) : j1;
    const float4* __restrict__ base = gsrc + off;
    for (int64_t jt = w0; jt < w1; jt += a.T) {
      const int cnt = (int)((w1 - jt < a.T) ? (w1 - jt) : a.T);
      const float q0 = base[jt].w;
      int same = 1;
      for (int k = lane; k < cnt; k += 64) same &= (base[jt + k].w == q0);
      const int uniform = __all(same);
      const int main = cnt & ~(kU - 1);
      float fx[R], fy[R], fz[R], fp[R], cx[R], cy[R], cz[R], cpc[R];
#pragma unroll
      for (int r = 0; r < R; ++r) { fx[r] = fy[r] = fz[r] = fp[r] = 0.f; cx[r] = cy[r] = cz[r] = cpc[r] = 0.f; }
      const float4* __restrict__ seg = base + jt;
      if (uniform) {
        pair_loop<R, PHI, KAHAN, true, kU, PBC>(seg, 0, main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
        pair_loop<R, PHI, KAHAN, true, 1, PBC>(seg, main, cnt - main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy,
                                               cz, cpc);
      } else {
        pair_loop<R, PHI, KAHAN, false, kU, PBC>(seg, 0, main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz,
                                                  cpc);
        pair_loop<R, PHI, KAHAN, false, 1, PBC>(seg, main, cnt - main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx,
                                                cy, cz, cpc);
      }
      const double qs = uniform ? (double)q0 : 1.0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ex[r] += (double)fx[r] * qs;
        ey[r] += (double)fy[r] * qs;
        ez[r] += (double)fz[r] * qs;
        if (PHI) ep[r] += (double)fp[r] * qs;
      }
    }
  } else
  for (int64_t jt = j0; jt < j1; jt += a.T) {
    const int cnt = (int)((j1 - jt < a.T) ? (j1 - jt) : a.T);
    const int cntp = (cnt + kU * WJ - 1) / (kU * WJ) * (kU * WJ);
    // Padding entries sit at 1e30: r^2 overflows to +inf, v_rsq_f32(+inf) = +0, so they add
    // exactly zero on both inner loops.  A tile whose sources all carry the same charge takes
    // the uniform loop, which factors the charge out of the pair term.  With periodic
    // boundaries the minimum image would bring such an entry close, so padding sits at the
    // origin with zero charge, and only a tile without padding takes the uniform loop.
    const float q0 = a.src[off + jt].w;
    int same = 1;
    __syncthreads();
    for (int k = tid; k < cntp; k += kBlock) {
      float4 v = PBC ? make_float4(0.f, 0.f, 0.f, 0.f) : make_float4(1e30f, 1e30f, 1e30f, 0.f);
      if (k < cnt) {
        v = a.src[off + jt + k];
        same &= (v.w == q0);
      }
      lds[k] = v;
    }
    const int uniform = __syncthreads_and(same) && (!PBC || cnt == cntp);
    const int per = cntp / WJ;
    const int kb = jw * per;
    float fx[R], fy[R], fz[R], fp[R], cx[R], cy[R], cz[R], cpc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { fx[r] = fy[r] = fz[r] = fp[r] = 0.f; cx[r] = cy[r] = cz[r] = cpc[r] = 0.f; }
    if (uniform)
      pair_loop<R, PHI, KAHAN, true, kU, PBC>(lds, kb, per, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
    else
      pair_loop<R, PHI, KAHAN, false, kU, PBC>(lds, kb, per, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
    const double qs = uniform ? (double)q0 : 1.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      ex[r] += (double)fx[r] * qs;
      ey[r] += (double)fy[r] * qs;
      ez[r] += (double)fz[r] * qs;
      if (PHI) ep[r] += (double)fp[r] * qs;
    }
  }

  // Combine the WJ waves that share these targets (fixed order), then write partials.
  constexpr int NC = PHI ? 4 : 3;
  if (WJ > 1) {
    __syncthreads();
    double* red = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      red[(0 * R + r) * kBlock + tid] = ex[r];
      red[(1 * R + r) * kBlock + tid] = ey[r];
      red[(2 * R + r) * kBlock + tid] = ez[r];
      if (PHI) red[(3 * R + r) * kBlock + tid] = ep[r];
    }
    __syncthreads();
    if (jw == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
        for (int q = 0; q < WJ; ++q) {
          const int o = (g * WJ + q) * 64 + lane;
          sx += red[(0 * R + r) * kBlock + o];
          sy += red[(1 * R + r) * kBlock + o];
          sz += red[(2 * R + r) * kBlock + o];
          if (PHI) sp += red[(3 * R + r) * kBlock + o];
        }
        ex[r] = sx; ey[r] = sy; ez[r] = sz; ep[r] = sp;
      }
    }
  }
  if (jw == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ii[r] < n) {
        const int64_t gs = off + ii[r];
        double* base = a.part + (int64_t)s * kComp * a.stride + gs;
        base[0] = ex[r];
        base[a.stride] = ey[r];
        base[2 * a.stride] = ez[r];
        if (PHI) base[3 * a.stride] = PBC ? ep[r] * (cp.box * (1.0 / 4294967296.0)) : ep[r];
      }
    }
  }
  (void)NC;
}

// ----------------------------------------------------------------------------- FP64 body
template <int R, int WJ, bool PHI, bool PBC>
__device__ void tile_f64(const ForceArgs<double4>& a, int t, double4* lds) {
  int c, ib, s;
  decode_tile(a.map, t, a.S, c, ib, s);
  const ClusterParams& cp = a.map.cp[c];
  const int64_t n = a.map.dyn[c].n_cur;
  const int64_t off = cp.off;
  constexpr int TG = 4 / WJ;
  constexpr int TI = TG * 64 * R;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;  // wave index, uniform
  const int g = w / WJ, jw = w % WJ;
  const int64_t i0 = (int64_t)ib * TI + (int64_t)g * 64 * R;

  const int64_t chunk = (n + a.S - 1) / a.S;
  const int64_t j0 = (int64_t)s * chunk;
  const int64_t j1 = (j0 + chunk < n) ? (j0 + chunk) : n;

  double xi[R], yi[R], zi[R];
  int64_t ii[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    ii[r] = i0 + r * 64 + lane;
    double4 p = (ii[r] < n) ? a.src[off + ii[r]] : make_double4(0.0, 0.0, 0.0, 0.0);
    xi[r] = p.x; yi[r] = p.y; zi[r] = p.z;
  }
  double ex[R], ey[R], ez[R], ep[R];
#pragma unroll
  for (int r = 0; r < R; ++r) { ex[r] = ey[r] = ez[r] = ep[r] = 0.0; }
  const double eps2 = a.eps2;
  const double L = PBC ? cp.box : 0.0;
  const double iL = PBC ? 1.0 / L : 0.0;

  for (int64_t jt = j0; jt < j1; jt += a.T) {
    const int cnt = (int)((j1 - jt < a.T) ? (j1 - jt) : a.T);
    const int cntp = (cnt + kU * WJ - 1) / (kU * WJ) * (kU * WJ);
    __syncthreads();
    for (int k = tid; k < cntp; k += kBlock)
      lds[k] = (k < cnt) ? a.src[off + jt + k] : make_double4(0.0, 0.0, 0.0, 0.0);
    __syncthreads();
    const int per = cntp / WJ;
    const int kb = jw * per;
    for (int k = kb; k < kb + per; k += kU) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const double4 sj = lds[k + u];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double dx = xi[r] - sj.x;
          double dy = yi[r] - sj.y;
          double dz = zi[r] - sj.z;
          if (PBC) {
            dx = min_image(dx, L, iL);
            dy = min_image(dy, L, iL);
            dz = min_image(dz, L, iL);
          }
          double r2 = __builtin_fma(dx, dx, eps2);
          r2 = __builtin_fma(dy, dy, r2);
          r2 = __builtin_fma(dz, dz, r2);
          const double inv = rsq64(r2);
          double qinv = sj.w * inv;
          const double sc = qinv * (inv * inv);
          ex[r] = __builtin_fma(sc, dx, ex[r]);
          ey[r] = __builtin_fma(sc, dy, ey[r]);
          ez[r] = __builtin_fma(sc, dz, ez[r]);
          if (PHI) {
            if (jt + k + u == ii[r]) qinv = 0.0;
            ep[r] += qinv;
          }
        }
      }
    }
  }

  if (WJ > 1) {
    __syncthreads();
    double* red = reinterpret_cast<double*>(lds);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      red[(0 * R + r) * kBlock + tid] = ex[r];
      red[(1 * R + r) * kBlock + tid] = ey[r];
      red[(2 * R + r) * kBlock + tid] = ez[r];
      if (PHI) red[(3 * R + r) * kBlock + tid] = ep[r];
    }
    __syncthreads();
    if (jw == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
        for (int q = 0; q < WJ; ++q) {
          const int o = (g * WJ + q) * 64 + lane;
          sx += red[(0 * R + r) * kBlock + o];
          sy += red[(1 * R + r) * kBlock + o];
          sz += red[(2 * R + r) * kBlock + o];
          if (PHI) sp += red[(3 * R + r) * kBlock + o];
        }
        ex[r] = sx; ey[r] = sy; ez[r] = sz; ep[r] = sp;
      }
    }
  }
  if (jw == 0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ii[r] < n) {
        const int64_t gs = off + ii[r];
        double* base = a.part + (int64_t)s * kComp * a.stride + gs;
        base[0] = ex[r];
        base[a.stride] = ey[r];
        base[2 * a.stride] = ez[r];
        if (PHI) base[3 * a.stride] = ep[r];
      }
    }
  }
}

// ----------------------------------------------------------------------------- pairs once
// Newton's third law: the pair term of (i, j) is the pair term of (j, i) with the sign of the
// separation flipped and the partner's charge, so one evaluation can serve both particles.
// A cluster's slots are cut into blocks of B slots.  The tile (I, J), I < J, takes every pair
// (i in block I, j in block J) once and produces E_i's part from block J and E_j's part from
// block I; the diagonal tile (I, I) takes all pairs of its block one-sided (the self pair adds
// exactly zero).  A thread block holds TG target groups of 64 R targets (R per lane), and the
// WJ waves of a group split the B sources: TG = 4/WJ (256 threads, B = (4/WJ) 64 R), or for the
// square shapes R = WJ >= 3, TG = 1 (64 R threads, B = 64 R).  A wave walks its sources in
// chunks of 64, staged twice in a row in its own LDS slice (structure of arrays x, y, z, q, so
// every read is a unit-stride dword access free of bank conflicts): at rotation k lane l meets
// source (l + k) mod 64 at index l + k, an immediate offset.  The reaction sums of the chunk's
// sources travel with the rotation in registers: lane l holds the running sum of source
// (l + k) mod 64, adds its terms, and hands it to lane l - 1 (DPP wave rotate by one lane), so
// after 64 rotations lane l holds source l's sum, accumulated in a fixed order (deterministic).
// Tiles of equal-charge sources or equal-charge targets factor the charge out of the pair term.
//
// Partial fields are rows of the pair type (FP32 rows for LC_FP32_ACC64, FP64 rows for
// LC_FP64), one per (block K, partner block m) of a cluster:
//   row (K, m), component d, local slot l:  n3part[n3_off + ((K M + m) 3 + d) B + l]
// written by exactly one tile.  M (rows per block) is fixed at creation; nb = ceil(n / B).
// A slot's field is the FP64 sum of its block's rows m = 0 .. nb - 1 in a fixed order, taken
// by the push kernel of the step (k_fold_push) or by k_fold_n3 into split 0 of the FP64
// partials (start, field snapshots).

// Pair arithmetic of the pair-once kernel: float (LC_FP32_ACC64) or double (LC_FP64).
// kFar places padding entries so far away that every term they take part in is exactly zero:
// FP32 r^2 overflows to +inf and v_rsq_f32(+inf) = +0; FP64 r^2 = 1e300 stays finite (the
// refined 1/sqrt needs a finite argument) and (1/r)^3 = 1e-450 underflows to zero.
template <typename T> struct N3Type;
template <> struct N3Type<float> {
  using V4 = float4;
  static constexpr float kFar = 1e30f;
};
template <> struct N3Type<double> {
  using V4 = double4;
  static constexpr double kFar = 1e150;
};

template <typename T>
struct N3Args {
  const typename N3Type<T>::V4* src;  // source records, global slot indexed
  T* part;                            // pair-once rows
  int M;                              // rows per block
  double eps2;
  int persistent;
  TileMap map;
  StepBegin begin;
};

__device__ inline float n3_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double n3_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ inline void decode_pair_tile(const TileMap& m, int t, int& c, int& I, int& J) {
  int lo = 0, hi = m.n_clusters - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (m.tile_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  c = m.order[lo];
  const int64_t local = t - m.tile_start[lo];
  // tiles of a cluster in J-major order: local = J (J + 1) / 2 + I, 0 <= I <= J
  // first guess from a single-precision square root (one VALU instruction rather than the
  // double-precision sequence); the two loops below make j exact
  int64_t j = (int64_t)((sqrtf(8.0f * (float)local + 1.0f) - 1.0f) * 0.5f);
  while (j * (j + 1) / 2 > local) --j;
  while ((j + 1) * (j + 2) / 2 <= local) ++j;
  J = (int)j;
  I = (int)(local - j * (j + 1) / 2);
}

// x from lane (l + 1) mod 64 for every lane l (DPP wave_rol:1).
__device__ inline float wave_rol1(float x) {
  // every lane of the wave has a source lane, so no "old" value is needed
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0x134, 0xf, 0xf, false));
}
__device__ inline double wave_rol1(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)b, 0x134, 0xf, 0xf, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(b >> 32), 0x134, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Orders the LDS traffic of one wave around a point where lanes read what other lanes wrote.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wave LDS slice: x, y, z, q arrays of the chunk twice (128 entries each) plus room for
// the prefetch of the rotation after the last one (up to 8 entries, read and discarded).
constexpr int kN3Slice = 136;
__host__ __device__ constexpr int n3_slices(int waves) { return waves * 4 * kN3Slice; }  // elements

// One chunk of 64 sources (sb: x, y, z, q arrays of the chunk twice, kN3Slice apart) against
// the lane's R targets.  US: all sources of the chunk carry one charge (factored out by the
// caller); UT: likewise for the targets of the wave.  JSIDE: also the reaction sums
// sum_r q_r s_r (r_i - r_j) of the chunk's sources, returned in (ax, ay, az) of lane l for
// source l.
// U rotations of the chunk from the register buffers (bx, by, bz, bq) holding their sources.
template <typename T, int R, int U, bool US, bool UT, bool JSIDE, bool PBC>
__device__ inline void n3_steps(const T* bx, const T* by, const T* bz, const T* bq, const T* xi, const T* yi,
                                const T* zi, const T* qi, T eps2f, T* fx, T* fy, T* fz, T& rx, T& ry, T& rz, T L,
                                T iL) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const T dx = pair_sep<T, PBC>(xi[r], bx[u], L, iL);
      const T dy = pair_sep<T, PBC>(yi[r], by[u], L, iL);
      const T dz = pair_sep<T, PBC>(zi[r], bz[u], L, iL);
      T r2 = n3_fma(dx, dx, eps2f);
      r2 = n3_fma(dy, dy, r2);
      r2 = n3_fma(dz, dz, r2);
      const T inv = n3_rsq(r2);
      const T r3 = inv * (inv * inv);
      const T si = US ? r3 : bq[u] * r3;
      fx[r] = n3_fma(si, dx, fx[r]);
      fy[r] = n3_fma(si, dy, fy[r]);
      fz[r] = n3_fma(si, dz, fz[r]);
      if (JSIDE) {
        const T sr = UT ? r3 : qi[r] * r3;
        rx = n3_fma(sr, dx, rx);
        ry = n3_fma(sr, dy, ry);
        rz = n3_fma(sr, dz, rz);
      }
    }
    if (JSIDE) {
      rx = wave_rol1(rx);
      ry = wave_rol1(ry);
      rz = wave_rol1(rz);
    }
  }
}

// Sources of rotations [k, k + U) into registers.
template <typename T, int U, bool US>
__device__ inline void n3_load(const T* sx, int k, T* bx, T* by, T* bz, T* bq) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    bx[u] = sx[k + u];
    by[u] = sx[kN3Slice + k + u];
    bz[u] = sx[2 * kN3Slice + k + u];
    if (!US) bq[u] = sx[3 * kN3Slice + k + u];
  }
}

// One chunk of 64 sources (sb: x, y, z, q arrays of the chunk twice, kN3Slice apart) against
// the lane's R targets.  US: all sources of the chunk carry one charge (factored out by the
// caller); UT: likewise for the targets of the wave.  JSIDE: also the reaction sums
// sum_r q_r s_r (r_i - r_j) of the chunk's sources, returned in (ax, ay, az) of lane l for
// source l.  Software pipelined over two register buffers: the sources of the next U
// rotations are read while the current U are used (the slice has kN3Slice >= 128 + U
// entries, so the read after the last rotation stays inside it).
template <typename T, int R, bool US, bool UT, bool JSIDE, bool PBC>
__device__ inline void n3_chunk(const T* sb, int lane, const T* xi, const T* yi, const T* zi, const T* qi, T eps2f,
                                T* fx, T* fy, T* fz, T& ax, T& ay, T& az, T L, T iL) {
  constexpr int U = (R >= 4 || sizeof(T) == 8) ? 2 : 4;  // rotations per register buffer
  static_assert(128 + U <= kN3Slice && 64 % (2 * U) == 0, "prefetch stays inside the wave's slice");
  const T* sx = sb + lane;
  T rx = 0, ry = 0, rz = 0;  // running sums of source (lane + k) mod 64
  T ax_[U], ay_[U], az_[U], aq_[U], bx_[U], by_[U], bz_[U], bq_[U];
  n3_load<T, U, US>(sx, 0, ax_, ay_, az_, aq_);
  for (int k0 = 0; k0 < 64; k0 += 2 * U) {
    n3_load<T, U, US>(sx, k0 + U, bx_, by_, bz_, bq_);
    n3_steps<T, R, U, US, UT, JSIDE, PBC>(ax_, ay_, az_, aq_, xi, yi, zi, qi, eps2f, fx, fy, fz, rx, ry, rz, L, iL);
    n3_load<T, U, US>(sx, k0 + 2 * U, ax_, ay_, az_, aq_);
    n3_steps<T, R, U, US, UT, JSIDE, PBC>(bx_, by_, bz_, bq_, xi, yi, zi, qi, eps2f, fx, fy, fz, rx, ry, rz, L, iL);
  }
  ax = rx;
  ay = ry;
  az = rz;
}

// Shapes: target groups per block are 4/WJ (blocks of 256 threads), except the square shapes
// R = WJ >= 3, which have one target group of 64 R targets and WJ waves, each wave one 64-source
// chunk (blocks of 64 R threads, B = 64 R).
__host__ __device__ constexpr int n3_groups(int R, int WJ) { return (R == WJ && R >= 3) ? 1 : 4 / WJ; }
__host__ __device__ constexpr int n3_waves(int R, int WJ) { return n3_groups(R, WJ) * WJ; }
__host__ __device__ constexpr int n3_block(int R, int WJ) { return n3_groups(R, WJ) * 64 * R; }

template <typename T, int R, int WJ, bool PBC>
__device__ void tile_n3(const N3Args<T>& a, int t, T* lds) {
  using V4 = typename N3Type<T>::V4;
  constexpr T kFar = N3Type<T>::kFar;
  constexpr int TG = n3_groups(R, WJ), NT = 64 * n3_waves(R, WJ), TGT = 64 * R, B = TG * TGT, PW = B / WJ,
                NCH = PW / 64;
  static_assert(PW % 64 == 0, "each wave takes whole chunks of 64 sources");
  int c, I, J;
  decode_pair_tile(a.map, t, c, I, J);
  const ClusterParams& cp = a.map.cp[c];
  const int64_t n = a.map.dyn[c].n_cur;
  const V4* __restrict__ src = a.src + cp.off;
  T* rows = a.part + cp.n3_off;
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int g = w / WJ, jw = w % WJ;
  const bool jside = (I != J);
  // rows exist only for blocks holding live slots (I <= J < nb <= M for a table built for n)
  const bool live = (int64_t)J * B < n && I <= J && J < a.M;
  T* sb = lds + w * 4 * kN3Slice;  // x, y, z, q arrays of the wave's chunk
  T* jres = lds + n3_slices(n3_waves(R, WJ));  // [TG][3][B] reaction sums of the block's sources
  T* ired = jres + TG * 3 * B;    // [WJ - 1][3][B] target sums of waves jw > 0

  const int64_t i0 = (int64_t)I * B + (int64_t)g * TGT;
  const bool tvalid = live && i0 < n;  // wave-uniform
  const T qT = tvalid ? src[i0].w : T(0);
  T xi[R], yi[R], zi[R], qi[R];
  int same_t = 1;
  if (i0 + TGT <= n) {
    // every target of the wave is a live slot: no padding
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const V4 p = src[i0 + r * 64 + lane];
      xi[r] = p.x; yi[r] = p.y; zi[r] = p.z; qi[r] = p.w;
      same_t &= (p.w == qT);
    }
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t ii = i0 + r * 64 + lane;
      if (ii < n) {
        const V4 p = src[ii];
        xi[r] = p.x; yi[r] = p.y; zi[r] = p.z; qi[r] = p.w;
        same_t &= (p.w == qT);
      } else if (PBC) {
        // the minimum image would bring a far entry close: zero charge at the origin instead
        xi[r] = yi[r] = zi[r] = 0;
        qi[r] = 0;
      } else {
        // far away: both sides add exactly zero (see N3Type)
        xi[r] = yi[r] = zi[r] = kFar;
        qi[r] = qT;
      }
    }
  }
  // periodic boundaries: the padding carries charge 0, so the target charge is factored out
  // only for a wave without padding
  const bool ut = __all(same_t) && (!PBC || i0 + TGT <= n);
  const T eps2f = pass_eps2<T, PBC>(a.eps2, cp.box);
  const T L = PBC ? (T)cp.box : T(0);
  const T iL = PBC ? T(1) / L : T(0);
  T ex[R], ey[R], ez[R];
#pragma unroll
  for (int r = 0; r < R; ++r) ex[r] = ey[r] = ez[r] = 0;

  if (tvalid) {
    for (int ch = 0; ch < NCH; ++ch) {
      const int64_t jb = (int64_t)J * B + jw * PW + ch * 64;
      if (jb >= n) break;
      const int64_t jj = jb + lane;
      const T qs0 = src[jb].w;
      V4 sv;
      bool us;
      if (jb + 64 <= n) {
        // a chunk of live sources only
        sv = src[jj];
        us = __all(sv.w == qs0);
      } else {
        if (jj < n) sv = src[jj];
        else if (PBC) { sv.x = 0; sv.y = 0; sv.z = 0; sv.w = 0; }
        else { sv.x = kFar; sv.y = kFar; sv.z = kFar; sv.w = 0; }
        us = PBC ? __all(jj < n && sv.w == qs0) : __all(jj >= n || sv.w == qs0);
      }
      sb[lane] = sv.x;
      sb[lane + 64] = sv.x;
      sb[kN3Slice + lane] = sv.y;
      sb[kN3Slice + lane + 64] = sv.y;
      sb[2 * kN3Slice + lane] = sv.z;
      sb[2 * kN3Slice + lane + 64] = sv.z;
      sb[3 * kN3Slice + lane] = sv.w;
      sb[3 * kN3Slice + lane + 64] = sv.w;
      wave_lds_sync();
      T cx[R], cy[R], cz[R], ax, ay, az;
#pragma unroll
      for (int r = 0; r < R; ++r) cx[r] = cy[r] = cz[r] = 0;
      if (jside) {
        if (us) {
          if (ut) n3_chunk<T, R, true, true, true, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
          else n3_chunk<T, R, true, false, true, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
        } else {
          if (ut) n3_chunk<T, R, false, true, true, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
          else n3_chunk<T, R, false, false, true, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
        }
      } else {
        if (us) n3_chunk<T, R, true, true, false, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
        else n3_chunk<T, R, false, true, false, PBC>(sb, lane, xi, yi, zi, qi, eps2f, cx, cy, cz, ax, ay, az, L, iL);
      }
      wave_lds_sync();
      const T fs = us ? qs0 : T(1);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        ex[r] = n3_fma(fs, cx[r], ex[r]);
        ey[r] = n3_fma(fs, cy[r], ey[r]);
        ez[r] = n3_fma(fs, cz[r], ez[r]);
      }
      if (jside) {
        // E_j = sum_i q_i (r_j - r_i) s_ij = -(reaction sum), charge factored when uniform
        const T js = ut ? -qT : T(-1);
        const int jl = jw * PW + ch * 64 + lane;
        jres[(g * 3 + 0) * B + jl] = js * ax;
        jres[(g * 3 + 1) * B + jl] = js * ay;
        jres[(g * 3 + 2) * B + jl] = js * az;
      }
      wave_lds_sync();  // every lane's reads of sb are done before the next chunk restages it
    }
  }
  __syncthreads();

  // Target side: the WJ waves of a group add up in a fixed order; row (I, J).
  if (WJ > 1) {
    if (jw > 0 && tvalid) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int l = g * TGT + r * 64 + lane;
        ired[((jw - 1) * 3 + 0) * B + l] = ex[r];
        ired[((jw - 1) * 3 + 1) * B + l] = ey[r];
        ired[((jw - 1) * 3 + 2) * B + l] = ez[r];
      }
    }
    __syncthreads();
    if (jw == 0 && tvalid) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int l = g * TGT + r * 64 + lane;
        for (int q = 0; q < WJ - 1; ++q) {
          ex[r] += ired[(q * 3 + 0) * B + l];
          ey[r] += ired[(q * 3 + 1) * B + l];
          ez[r] += ired[(q * 3 + 2) * B + l];
        }
      }
    }
  }
  if (jw == 0 && tvalid) {
    T* row = rows + (int64_t)((int64_t)I * a.M + J) * 3 * B;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int l = g * TGT + r * 64 + lane;
      if ((int64_t)I * B + l < n) {
        row[l] = ex[r];
        row[B + l] = ey[r];
        row[2 * B + l] = ez[r];
      }
    }
  }
  // Source side: the target groups add up in a fixed order; row (J, I).
  if (jside && live) {
    T* row = rows + (int64_t)((int64_t)J * a.M + I) * 3 * B;
    for (int jl = tid; jl < B; jl += NT) {
      if ((int64_t)J * B + jl >= n) break;
      T sx = 0, sy = 0, sz = 0;
      for (int q = 0; q < TG; ++q) {
        if ((int64_t)I * B + (int64_t)q * TGT >= n) break;
        sx += jres[(q * 3 + 0) * B + jl];
        sy += jres[(q * 3 + 1) * B + jl];
        sz += jres[(q * 3 + 2) * B + jl];
      }
      row[jl] = sx;
      row[B + jl] = sy;
      row[2 * B + jl] = sz;
    }
  }
}

// Row sums of the pair-once pass: a block of kFoldWaves waves takes 64 consecutive global
// slots; wave w adds rows m = w, w + kFoldWaves, ... (coalesced across the lanes), and wave 0 combines
// the partial sums in order.  Writes E into components 0..2 of split 0 for live slots of
// active clusters.
template <typename Tr>
__global__ __launch_bounds__(64 * kFoldWaves) void k_fold_n3(DevState s, RunConst rc, int B) {
  __shared__ double red[kFoldWaves - 1][3][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t g = (int64_t)blockIdx.x * 64 + lane;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  bool live = false;
  if (g < rc.n_total) {
    const int c = wave_cluster(s, (int64_t)blockIdx.x * 64);
    live = s.dyn[c].active && g - s.cp[c].off < s.dyn[c].n_sched;
    if (live) n3_row_partial<Tr>(s, rc, B, g, c, w, kFoldWaves, e0, e1, e2);
  }
  if (w > 0) {
    red[w - 1][0][lane] = e0;
    red[w - 1][1][lane] = e1;
    red[w - 1][2][lane] = e2;
  }
  __syncthreads();
  if (w == 0 && live) {
    for (int q = 0; q < kFoldWaves - 1; ++q) {
      e0 += red[q][0][lane];
      e1 += red[q][1][lane];
      e2 += red[q][2][lane];
    }
    s.part[g] = e0;
    s.part[rc.n_total + g] = e1;
    s.part[2 * rc.n_total + g] = e2;
  }
}

// ----------------------------------------------------------------------------- kernels
// Occupancy the register allocation aims at: 5 waves per SIMD for FP32 pairs (85 VGPRs at
// R = 4, no spills; 4 from R = 6), 3 for FP64 pairs (twice the registers per value; 2 from R = 5).
template <typename T, int R, int WJ, bool PBC>
__global__ __launch_bounds__(64 * n3_waves(R, WJ))
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? (R >= 5 ? 2 : 3) : (R >= 6 ? 4 : 5))))
void k_force_n3(N3Args<T> a) {
  extern __shared__ __align__(16) unsigned char lds_n3_raw[];
  T* lds_n3 = reinterpret_cast<T*>(lds_n3_raw);
  if (a.begin.on && blockIdx.x == 0 && threadIdx.x < 64) begin_step_wave(a.begin);
  const int total = *a.map.tile_total;
  if (!a.persistent) {
    // one tile per block when the grid covers the tiles, else a block-strided walk over them
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
      if (t != (int)blockIdx.x) __syncthreads();
      tile_n3<T, R, WJ, PBC>(a, t, lds_n3);
    }
    return;
  }
  __shared__ int sh_t;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_t = atomicAdd(a.map.queue, 1);
    __syncthreads();
    const int t = sh_t;
    if (t >= total) break;
    tile_n3<T, R, WJ, PBC>(a, t, lds_n3);
  }
}

template <int R, int WJ, bool PHI, bool KAHAN, bool SCALAR, bool PBC>
__global__ __launch_bounds__(kBlock) void k_force_f32(ForceArgs<float4> a, const float4* __restrict__ gsrc) {
  extern __shared__ float4 lds32[];
  if (a.begin.on && blockIdx.x == 0 && threadIdx.x < 64) begin_step_wave(a.begin);
  const int total = *a.map.tile_total;
  if (!a.persistent) {
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
      if (t != (int)blockIdx.x) __syncthreads();
      tile_f32<R, WJ, PHI, KAHAN, SCALAR, PBC>(a, gsrc, t, lds32);
    }
    return;
  }
  __shared__ int sh_t;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_t = atomicAdd(a.map.queue, 1);
    __syncthreads();
    const int t = sh_t;
    if (t >= total) break;
    tile_f32<R, WJ, PHI, KAHAN, SCALAR, PBC>(a, gsrc, t, lds32);
  }
}

template <int R, int WJ, bool PHI, bool PBC>
__global__ __launch_bounds__(kBlock) void k_force_f64(ForceArgs<double4> a) {
  extern __shared__ double4 lds64[];
  if (a.begin.on && blockIdx.x == 0 && threadIdx.x < 64) begin_step_wave(a.begin);
  const int total = *a.map.tile_total;
  if (!a.persistent) {
    for (int t = blockIdx.x; t < total; t += gridDim.x) {
      if (t != (int)blockIdx.x) __syncthreads();
      tile_f64<R, WJ, PHI, PBC>(a, t, lds64);
    }
    return;
  }
  __shared__ int sh_t;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_t = atomicAdd(a.map.queue, 1);
    __syncthreads();
    const int t = sh_t;
    if (t >= total) break;
    tile_f64<R, WJ, PHI, PBC>(a, t, lds64);
  }
}

size_t force_lds_bytes(int precision, const ForceTiling& ft, bool phi) {
  const size_t src = (precision == LC_FP64) ? sizeof(double4) : sizeof(float4);
  size_t tile = (ft.scalar_src && precision != LC_FP64) ? 0 : (size_t)(ft.T + kU * ft.WJ) * src;
  size_t red = (ft.WJ > 1) ? (size_t)(phi ? 4 : 3) * ft.R * kBlock * sizeof(double) : 0;
  return tile > red ? tile : red;
}

// pbc: minimum-image separations (periodic boundaries); not with Kahan sums.
template <int R, int WJ>
hipError_t dispatch_f32(const ForceArgs<float4>& a, bool phi, int kahan, int scalar, bool pbc, int grid, size_t lds,
                        hipStream_t st) {
  if (pbc) {
    if (kahan) return hipErrorInvalidValue;
    if (scalar) {
      if (phi) k_force_f32<R, WJ, true, false, true, true><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, false, true, true><<<grid, kBlock, lds, st>>>(a, a.src);
    } else {
      if (phi) k_force_f32<R, WJ, true, false, false, true><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, false, false, true><<<grid, kBlock, lds, st>>>(a, a.src);
    }
    return hipGetLastError();
  }
  if (scalar) {
    if (kahan) {
      if (phi) k_force_f32<R, WJ, true, true, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, true, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
    } else {
      if (phi) k_force_f32<R, WJ, true, false, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, false, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
    }
  } else if (kahan) {
    if (phi) k_force_f32<R, WJ, true, true, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
    else k_force_f32<R, WJ, false, true, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
  } else {
    if (phi) k_force_f32<R, WJ, true, false, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
    else k_force_f32<R, WJ, false, false, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
  }
  return hipGetLastError();
}

template <int R, int WJ>
hipError_t dispatch_f64(const ForceArgs<double4>& a, bool phi, bool pbc, int grid, size_t lds, hipStream_t st) {
  if (pbc) {
    if (phi) k_force_f64<R, WJ, true, true><<<grid, kBlock, lds, st>>>(a);
    else k_force_f64<R, WJ, false, true><<<grid, kBlock, lds, st>>>(a);
  } else {
    if (phi) k_force_f64<R, WJ, true, false><<<grid, kBlock, lds, st>>>(a);
    else k_force_f64<R, WJ, false, false><<<grid, kBlock, lds, st>>>(a);
  }
  return hipGetLastError();
}

// Pair-once shapes: whole 64-source chunks per wave, blocks of 128..512 slots, and every shape
// also valid for the regular kernels (which take the steps that need the potential).
bool n3_shape_ok(int R, int WJ) {
  return (WJ == 1 && (R == 1 || R == 2)) || (WJ == 2 && (R == 1 || R == 2 || R == 4)) ||
         (R == WJ && R >= 3 && R <= 6);
}

size_t n3_lds_bytes(const ForceTiling& ft, size_t elem) {
  const size_t B = (size_t)n3_block(ft.R, ft.WJ);
  return elem * ((size_t)n3_slices(n3_waves(ft.R, ft.WJ)) + (size_t)n3_groups(ft.R, ft.WJ) * 3 * B +
                 (size_t)(ft.WJ - 1) * 3 * B);
}

size_t n3_elem(int precision) { return precision == LC_FP64 ? sizeof(double) : sizeof(float); }

// Workgroups of the pair-once kernel one CU holds at once (occupancy), cached per shape.
// Pair-once shapes and their kernels: key WJ * 16 + R.
#define LC_N3_SHAPES(X)                                                                          \
  X(1, 1) X(2, 1) X(1, 2) X(2, 2) X(4, 2) X(3, 3) X(4, 4) X(5, 5) X(6, 6)

template <typename T>
int n3_resident_t(const ForceTiling& ft) {
  const size_t lds = n3_lds_bytes(ft, sizeof(T));
  const int threads = 64 * n3_waves(ft.R, ft.WJ);
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (ft.WJ * 16 + ft.R) {
#define LC_N3_OCC(R_, WJ_)                                                                         \
  case WJ_ * 16 + R_:                                                                               \
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_force_n3<T, R_, WJ_, false>, threads, lds); break;
    LC_N3_SHAPES(LC_N3_OCC)
#undef LC_N3_OCC
    default: break;
  }
  return (e == hipSuccess && nb > 0) ? nb : 4;
}

int n3_resident_per_cu(int precision, const ForceTiling& ft) {
  static int cache[2][8][8] = {};
  int& v = cache[precision == LC_FP64 ? 1 : 0][ft.R & 7][ft.WJ & 7];
  if (v > 0) return v;
  v = (precision == LC_FP64) ? n3_resident_t<double>(ft) : n3_resident_t<float>(ft);
  return v;
}

template <typename T>
hipError_t launch_n3(const ForceTiling& ft, const N3Args<T>& a, int grid, bool pbc, hipStream_t st,
                     hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
  const size_t lds = n3_lds_bytes(ft, sizeof(T));
  const int threads = 64 * n3_waves(ft.R, ft.WJ);
  switch (ft.WJ * 16 + ft.R) {
#define LC_N3_LAUNCH(R_, WJ_)                                                            \
  case WJ_ * 16 + R_:                                                                    \
    if (pbc) launch_timed(k_force_n3<T, R_, WJ_, true>, dim3(grid), dim3(threads), lds, st, e0, e1, a); \
    else launch_timed(k_force_n3<T, R_, WJ_, false>, dim3(grid), dim3(threads), lds, st, e0, e1, a);   \
    break;
    LC_N3_SHAPES(LC_N3_LAUNCH)
#undef LC_N3_LAUNCH
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define LC_WJ_SWITCH(R, FN, ...)                                   \
  switch (ft.WJ) {                                                  \
    case 1: return FN<R, 1>(__VA_ARGS__);                           \
    case 2: return FN<R, 2>(__VA_ARGS__);                           \
    case 4: return FN<R, 4>(__VA_ARGS__);                           \
    default: return hipErrorInvalidValue;                           \
  }

hipError_t launch_generic(int precision, const ForceTiling& ft, const TileMap& map, const void* src,
                          double* part, int64_t stride, double eps2, bool phi, bool pbc, int grid, hipStream_t st,
                          const StepBegin& sb = StepBegin{}) {
  const size_t lds = force_lds_bytes(precision, ft, phi);
  if (precision == LC_FP64) {
    ForceArgs<double4> a{(const double4*)src, part, stride, eps2, ft.T, ft.S, ft.persistent, map, sb};
    switch (ft.R) {
      case 1: LC_WJ_SWITCH(1, dispatch_f64, a, phi, pbc, grid, lds, st)
      case 2: LC_WJ_SWITCH(2, dispatch_f64, a, phi, pbc, grid, lds, st)
      case 4: LC_WJ_SWITCH(4, dispatch_f64, a, phi, pbc, grid, lds, st)
      default: return hipErrorInvalidValue;
    }
  }
  ForceArgs<float4> a{(const float4*)src, part, stride, eps2, ft.T, ft.S, ft.persistent, map, sb};
  const int kahan = (precision == LC_FP32_KAHAN);
  switch (ft.R) {
    case 1: LC_WJ_SWITCH(1, dispatch_f32, a, phi, kahan, ft.scalar_src, pbc, grid, lds, st)
    case 2: LC_WJ_SWITCH(2, dispatch_f32, a, phi, kahan, ft.scalar_src, pbc, grid, lds, st)
    case 4: LC_WJ_SWITCH(4, dispatch_f32, a, phi, kahan, ft.scalar_src, pbc, grid, lds, st)
    case 8:
      if (ft.WJ != 1) return hipErrorInvalidValue;
      return dispatch_f32<8, 1>(a, phi, kahan, ft.scalar_src, pbc, grid, lds, st);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------------------------------- standalone field
// Workspace: [ClusterParams][ClusterDyn][ints: tile_start(2), order(1), tile_total, queue]
//            [sources n][partials S*4*n]
struct FieldWs {
  ClusterParams* cp;
  ClusterDyn* dyn;
  int32_t* ints;
  void* src;
  double* part;      // split partials (regular kernels) or pair-once rows (newton3), as floats
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

FieldWs carve_field_ws(void* work, int precision, int64_t n, const ForceTiling& ft) {
  char* p = (char*)work;
  FieldWs w;
  w.cp = (ClusterParams*)p; p += align256(sizeof(ClusterParams));
  w.dyn = (ClusterDyn*)p; p += align256(sizeof(ClusterDyn));
  w.ints = (int32_t*)p; p += 256;
  w.src = p; p += align256((size_t)n * (precision == LC_FP64 ? sizeof(double4) : sizeof(float4)));
  w.part = (double*)p;
  return w;
}

__global__ void k_field_setup(FieldWs w, int64_t n, int i_blocks, int tiles) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ClusterParams cp = {};
    cp.off = 0;
    cp.cap = n;
    cp.n3_off = 0;
    *w.cp = cp;
    ClusterDyn d = {};
    d.n_cur = n;
    d.i_blocks = i_blocks;
    d.n_tiles = tiles;
    d.active = 1;
    *w.dyn = d;
    w.ints[0] = 0;
    w.ints[1] = d.n_tiles;
    w.ints[2] = 0;
    w.ints[3] = d.n_tiles;
    w.ints[4] = 0;
  }
}

template <typename Src>
__global__ void k_pack_sources(const double* xyzq, int64_t n, Src* out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Src v;
  v.x = xyzq[i];
  v.y = xyzq[n + i];
  v.z = xyzq[2 * n + i];
  v.w = xyzq[3 * n + i];
  out[i] = v;
}

__global__ void k_sum_partials(const double* part, int64_t n, int S, double* E, double* phi) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0, p = 0.0;
  for (int s = 0; s < S; ++s) {
    const double* b = part + (int64_t)s * kComp * n + i;
    e0 += b[0];
    e1 += b[n];
    e2 += b[2 * n];
    if (phi) p += b[3 * n];
  }
  E[i] = e0;
  E[n + i] = e1;
  E[2 * n + i] = e2;
  if (phi) phi[i] = p;
}

// Field of the standalone call from pair-once rows (M = nb rows per block).
template <typename Tr>
__global__ void k_sum_n3(const Tr* rows, int64_t n, int B, double* E) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t K = i / B, l = i - K * B;
  const int64_t nb = (n + B - 1) / B;
  const Tr* r = rows + K * nb * 3 * B + l;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  for (int64_t m = 0; m < nb; ++m, r += 3 * (int64_t)B) {
    e0 += (double)r[0];
    e1 += (double)r[B];
    e2 += (double)r[2 * B];
  }
  E[i] = e0;
  E[n + i] = e1;
  E[2 * n + i] = e2;
}

}  // namespace

int force_tile_targets(const ForceTiling& ft) { return (4 / ft.WJ) * 64 * ft.R; }

int n3_block_size(const ForceTiling& ft) { return n3_block(ft.R, ft.WJ); }

int n3_persistent_grid(int precision, const ForceTiling& ft, int64_t tiles, int cus) {
  // as many workgroups as fit at once, trimmed so that every one of them takes the same
  // number of tiles (within one) in the same number of rounds
  const int64_t pmax = std::max<int64_t>(1, (int64_t)cus * n3_resident_per_cu(precision, ft));
  const int64_t t = std::max<int64_t>(tiles, 1);
  const int64_t rounds = (t + pmax - 1) / pmax;
  return (int)((t + rounds - 1) / rounds);
}

int64_t n3_tiles(int64_t n, int B) {
  const int64_t nb = (n + B - 1) / B;
  return nb * (nb + 1) / 2;
}

// The one-sided tiling a pair-once tiling's diagnostic steps run with: its own fields when
// the one-sided kernels have that (R, WJ), else R = 1 (FP32) or 2 (FP64), WJ = 4.  With
// scalar sources (FP32) it is R = 1, WJ = 4, the fastest scalar-source form (on the 20k Ar
// cluster the one-sided field pass takes 127 us there against 148 us at R = 4, WJ = 4).
ForceTiling regular_tiling(int precision, const ForceTiling& ft) {
  ForceTiling r = ft;
  r.newton3 = 0;
  const bool wj_ok = ft.WJ == 1 || ft.WJ == 2 || ft.WJ == 4;
  const bool r_ok = ft.R == 1 || ft.R == 2 || ft.R == 4 || (ft.R == 8 && precision != LC_FP64 && ft.WJ == 1);
  if (!(wj_ok && r_ok) || (ft.scalar_src && precision != LC_FP64)) {
    r.R = (precision == LC_FP64) ? 2 : 1;
    r.WJ = 4;
  }
  return r;
}

bool force_tiling_valid(int precision, const ForceTiling& ft) {
  if (ft.newton3) {
    if (precision == LC_FP32_KAHAN || !n3_shape_ok(ft.R, ft.WJ)) return false;
    if (n3_lds_bytes(ft, n3_elem(precision)) > 64 * 1024) return false;
    return force_tiling_valid(precision, regular_tiling(precision, ft));
  }
  bool r_ok = ft.R == 1 || ft.R == 2 || ft.R == 4 || (ft.R == 8 && precision != LC_FP64 && ft.WJ == 1);
  bool wj_ok = ft.WJ == 1 || ft.WJ == 2 || ft.WJ == 4;
  bool t_ok = ft.T >= 64 && ft.T <= 4096 && (ft.T % 64) == 0;
  if (ft.scalar_src && precision == LC_FP64) return false;  // scalar source path is FP32 only
  bool s_ok = ft.S >= 1 && ft.S <= 64;
  if (!(r_ok && wj_ok && t_ok && s_ok)) return false;
  return force_lds_bytes(precision, ft, true) <= 64 * 1024;
}

hipError_t launch_force(const DevState& s, const RunConst& rc, int precision, const ForceTiling& ft,
                        bool want_phi, bool pbc, int grid_blocks, hipStream_t st, bool fold_n3, bool begin_step,
                        hipEvent_t e0, hipEvent_t e1) {
  TileMap map{s.tile_start, s.order, s.cp, s.dyn, s.tile_total, s.queue, rc.n_clusters};
  if (begin_step && (ft.persistent || !s.laser_tab)) return hipErrorInvalidValue;
  const StepBegin sb{s.dyn, s.cp, s.step, s.laser_tab, s.laser_tab0, rc.n_clusters, begin_step ? 1 : 0};
  if (ft.newton3 && !want_phi) {
    if (precision == LC_FP32_KAHAN || rc.n3_rows <= 0) return hipErrorInvalidValue;
    hipError_t e;
    const int fb = (int)((rc.n_total + 63) / 64);
    if (precision == LC_FP64) {
      N3Args<double> a{s.posq, (double*)s.n3part, rc.n3_rows, rc.eps2, ft.persistent, map, sb};
      e = launch_n3(ft, a, grid_blocks, pbc, st, e0, e1);
      if (e != hipSuccess || !fold_n3) return e;
      k_fold_n3<double><<<fb, 64 * kFoldWaves, 0, st>>>(s, rc, n3_block(ft.R, ft.WJ));
    } else {
      N3Args<float> a{s.pos4, (float*)s.n3part, rc.n3_rows, rc.eps2, ft.persistent, map, sb};
      e = launch_n3(ft, a, grid_blocks, pbc, st, e0, e1);
      if (e != hipSuccess || !fold_n3) return e;
      k_fold_n3<float><<<fb, 64 * kFoldWaves, 0, st>>>(s, rc, n3_block(ft.R, ft.WJ));
    }
    return hipGetLastError();
  }
  const void* src = (precision == LC_FP64) ? (const void*)s.posq : (const void*)s.pos4;
  const ForceTiling fr = ft.newton3 ? regular_tiling(precision, ft) : ft;
  if (begin_step && fr.persistent) return hipErrorInvalidValue;
  return launch_generic(precision, fr, map, src, s.part, rc.n_total, rc.eps2, want_phi, pbc, grid_blocks, st, sb);
}

// ----------------------------------------------------------------------------- allocation-free field
// Workspace of lc_field_static: a file-scope device array of LC_FIELD_STATIC_MAX_BYTES that each
// device holds for the life of the process.  On the host its name is only a stand-in for the
// symbol: host code uses the device address hipGetSymbolAddress returns for the current device,
// looked up once per device (each device has its own copy at its own address).
namespace {
static __device__ __align__(256) unsigned char scratch[LC_FIELD_STATIC_MAX_BYTES];
constexpr int kScratchDevices = 64;
}  // namespace

hipError_t field_scratch(void** out) {
  static std::mutex mu;
  static void* ptr[kScratchDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p || ((uintptr_t)p & 255) != 0) return hipErrorInvalidSymbol;
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return hipSuccess;
}

size_t field_workspace_bytes(int precision, int64_t n, const ForceTiling& ft) {
  size_t b = align256(sizeof(ClusterParams)) + align256(sizeof(ClusterDyn)) + 256;
  b += align256((size_t)n * (precision == LC_FP64 ? sizeof(double4) : sizeof(float4)));
  if (ft.newton3) {
    const size_t B = (size_t)n3_block(ft.R, ft.WJ);
    const size_t nb = ((size_t)n + B - 1) / B;
    b += align256(nb * nb * 3 * B * n3_elem(precision));
  } else {
    b += align256((size_t)ft.S * kComp * (size_t)n * sizeof(double));
  }
  return b;
}

hipError_t launch_field_standalone(int precision, int64_t n, const double* xyzq, double eps2, double* E,
                                   double* phi, void* work, const ForceTiling& ft, hipStream_t st) {
  if (n == 0) return hipSuccess;
  FieldWs w = carve_field_ws(work, precision, n, ft);
  const int TI = ft.newton3 ? n3_block(ft.R, ft.WJ) : force_tile_targets(ft);
  const int ib = (int)((n + TI - 1) / TI);
  const int64_t tiles = ft.newton3 ? (int64_t)ib * (ib + 1) / 2 : (int64_t)ib * ft.S;
  if (tiles > std::numeric_limits<int32_t>::max()) return hipErrorInvalidValue;
  k_field_setup<<<1, 64, 0, st>>>(w, n, ib, (int)tiles);
  const int pb = (int)((n + kBlock - 1) / kBlock);
  if (precision == LC_FP64) k_pack_sources<double4><<<pb, kBlock, 0, st>>>(xyzq, n, (double4*)w.src);
  else k_pack_sources<float4><<<pb, kBlock, 0, st>>>(xyzq, n, (float4*)w.src);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TileMap map{w.ints, w.ints + 2, w.cp, w.dyn, w.ints + 3, w.ints + 4, 1};
  int grid = (int)tiles;
  if (ft.persistent) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int pg = cus * 8;
    grid = grid < pg ? grid : pg;
  }
  if (ft.newton3) {
    if (phi) return hipErrorInvalidValue;
    if (precision == LC_FP64) {
      N3Args<double> a{(const double4*)w.src, (double*)w.part, ib, eps2, ft.persistent, map, StepBegin{}};
      e = launch_n3(ft, a, grid, false, st);
      if (e != hipSuccess) return e;
      k_sum_n3<double><<<pb, kBlock, 0, st>>>((const double*)w.part, n, TI, E);
    } else {
      N3Args<float> a{(const float4*)w.src, (float*)w.part, ib, eps2, ft.persistent, map, StepBegin{}};
      e = launch_n3(ft, a, grid, false, st);
      if (e != hipSuccess) return e;
      k_sum_n3<float><<<pb, kBlock, 0, st>>>((const float*)w.part, n, TI, E);
    }
    return hipGetLastError();
  }
  e = launch_generic(precision, ft, map, w.src, w.part, n, eps2, phi != nullptr, false, grid, st);
  if (e != hipSuccess) return e;
  k_sum_partials<<<pb, kBlock, 0, st>>>(w.part, n, ft.S, E, phi);
  return hipGetLastError();
}

}  // namespace lc

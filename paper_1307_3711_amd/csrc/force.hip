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

// ----------------------------------------------------------------------------- FP32 pair loop
// Sources [kb, kb + per) of the LDS tile against the lane's R targets.  UNIFORM: every source
// has the same charge q0 and the caller multiplies the sums by it (q r^-3 costs one multiply
// less per pair).  PHI: also the potential, with the self pair masked out by index.
// src is an LDS tile, or a global source array read with wave-uniform indices (the compiler
// then issues scalar loads and the pair arithmetic takes SGPR operands).  The sums and the
// Kahan compensations (cx..cpc) accumulate onto the caller's registers.
template <int R, bool PHI, bool KAHAN, bool UNIFORM, int U, typename P>
__device__ inline void pair_loop(P src, int kb, int per, int64_t jt, const int64_t* ii, const float* xi,
                                 const float* yi, const float* zi, float eps2f, float* fx, float* fy, float* fz,
                                 float* fp, float* cx, float* cy, float* cz, float* cpc) {
  for (int k = kb; k < kb + per; k += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const float4 sj = src[k + u];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float dx = xi[r] - sj.x;
        const float dy = yi[r] - sj.y;
        const float dz = zi[r] - sj.z;
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
template <int R, int WJ, bool PHI, bool KAHAN, bool SCALAR>
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
  const float eps2f = (float)a.eps2;

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
        pair_loop<R, PHI, KAHAN, true, kU>(seg, 0, main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
        pair_loop<R, PHI, KAHAN, true, 1>(seg, main, cnt - main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz,
                                          cpc);
      } else {
        pair_loop<R, PHI, KAHAN, false, kU>(seg, 0, main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
        pair_loop<R, PHI, KAHAN, false, 1>(seg, main, cnt - main, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz,
                                           cpc);
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
    // the uniform loop, which factors the charge out of the pair term.
    const float q0 = a.src[off + jt].w;
    int same = 1;
    __syncthreads();
    for (int k = tid; k < cntp; k += kBlock) {
      float4 v = make_float4(1e30f, 1e30f, 1e30f, 0.f);
      if (k < cnt) {
        v = a.src[off + jt + k];
        same &= (v.w == q0);
      }
      lds[k] = v;
    }
    const int uniform = __syncthreads_and(same);
    const int per = cntp / WJ;
    const int kb = jw * per;
    float fx[R], fy[R], fz[R], fp[R], cx[R], cy[R], cz[R], cpc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { fx[r] = fy[r] = fz[r] = fp[r] = 0.f; cx[r] = cy[r] = cz[r] = cpc[r] = 0.f; }
    if (uniform)
      pair_loop<R, PHI, KAHAN, true, kU>(lds, kb, per, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
    else
      pair_loop<R, PHI, KAHAN, false, kU>(lds, kb, per, jt, ii, xi, yi, zi, eps2f, fx, fy, fz, fp, cx, cy, cz, cpc);
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
        if (PHI) base[3 * a.stride] = ep[r];
      }
    }
  }
  (void)NC;
}

// ----------------------------------------------------------------------------- FP64 body
template <int R, int WJ, bool PHI>
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
          const double dx = xi[r] - sj.x;
          const double dy = yi[r] - sj.y;
          const double dz = zi[r] - sj.z;
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

// ----------------------------------------------------------------------------- kernels
template <int R, int WJ, bool PHI, bool KAHAN, bool SCALAR>
__global__ __launch_bounds__(kBlock) void k_force_f32(ForceArgs<float4> a, const float4* __restrict__ gsrc) {
  extern __shared__ float4 lds32[];
  const int total = *a.map.tile_total;
  if (!a.persistent) {
    if ((int)blockIdx.x < total) tile_f32<R, WJ, PHI, KAHAN, SCALAR>(a, gsrc, blockIdx.x, lds32);
    return;
  }
  __shared__ int sh_t;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_t = atomicAdd(a.map.queue, 1);
    __syncthreads();
    const int t = sh_t;
    if (t >= total) break;
    tile_f32<R, WJ, PHI, KAHAN, SCALAR>(a, gsrc, t, lds32);
  }
}

template <int R, int WJ, bool PHI>
__global__ __launch_bounds__(kBlock) void k_force_f64(ForceArgs<double4> a) {
  extern __shared__ double4 lds64[];
  const int total = *a.map.tile_total;
  if (!a.persistent) {
    if ((int)blockIdx.x < total) tile_f64<R, WJ, PHI>(a, blockIdx.x, lds64);
    return;
  }
  __shared__ int sh_t;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) sh_t = atomicAdd(a.map.queue, 1);
    __syncthreads();
    const int t = sh_t;
    if (t >= total) break;
    tile_f64<R, WJ, PHI>(a, t, lds64);
  }
}

size_t force_lds_bytes(int precision, const ForceTiling& ft, bool phi) {
  const size_t src = (precision == LC_FP64) ? sizeof(double4) : sizeof(float4);
  size_t tile = (ft.scalar_src && precision != LC_FP64) ? 0 : (size_t)(ft.T + kU * ft.WJ) * src;
  size_t red = (ft.WJ > 1) ? (size_t)(phi ? 4 : 3) * ft.R * kBlock * sizeof(double) : 0;
  return tile > red ? tile : red;
}

template <int R, int WJ>
hipError_t dispatch_f32(const ForceArgs<float4>& a, bool phi, int kahan, int scalar, int grid, size_t lds,
                        hipStream_t st) {
  if (scalar) {
    if (kahan) {
      if (phi) k_force_f32<R, WJ, true, true, true><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, true, true><<<grid, kBlock, lds, st>>>(a, a.src);
    } else {
      if (phi) k_force_f32<R, WJ, true, false, true><<<grid, kBlock, lds, st>>>(a, a.src);
      else k_force_f32<R, WJ, false, false, true><<<grid, kBlock, lds, st>>>(a, a.src);
    }
  } else if (kahan) {
    if (phi) k_force_f32<R, WJ, true, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
    else k_force_f32<R, WJ, false, true, false><<<grid, kBlock, lds, st>>>(a, a.src);
  } else {
    if (phi) k_force_f32<R, WJ, true, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
    else k_force_f32<R, WJ, false, false, false><<<grid, kBlock, lds, st>>>(a, a.src);
  }
  return hipGetLastError();
}

template <int R, int WJ>
hipError_t dispatch_f64(const ForceArgs<double4>& a, bool phi, int grid, size_t lds, hipStream_t st) {
  if (phi) k_force_f64<R, WJ, true><<<grid, kBlock, lds, st>>>(a);
  else k_force_f64<R, WJ, false><<<grid, kBlock, lds, st>>>(a);
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
                          double* part, int64_t stride, double eps2, bool phi, int grid, hipStream_t st) {
  const size_t lds = force_lds_bytes(precision, ft, phi);
  if (precision == LC_FP64) {
    ForceArgs<double4> a{(const double4*)src, part, stride, eps2, ft.T, ft.S, ft.persistent, map};
    switch (ft.R) {
      case 1: LC_WJ_SWITCH(1, dispatch_f64, a, phi, grid, lds, st)
      case 2: LC_WJ_SWITCH(2, dispatch_f64, a, phi, grid, lds, st)
      case 4: LC_WJ_SWITCH(4, dispatch_f64, a, phi, grid, lds, st)
      default: return hipErrorInvalidValue;
    }
  }
  ForceArgs<float4> a{(const float4*)src, part, stride, eps2, ft.T, ft.S, ft.persistent, map};
  const int kahan = (precision == LC_FP32_KAHAN);
  switch (ft.R) {
    case 1: LC_WJ_SWITCH(1, dispatch_f32, a, phi, kahan, ft.scalar_src, grid, lds, st)
    case 2: LC_WJ_SWITCH(2, dispatch_f32, a, phi, kahan, ft.scalar_src, grid, lds, st)
    case 4: LC_WJ_SWITCH(4, dispatch_f32, a, phi, kahan, ft.scalar_src, grid, lds, st)
    case 8:
      if (ft.WJ != 1) return hipErrorInvalidValue;
      return dispatch_f32<8, 1>(a, phi, kahan, ft.scalar_src, grid, lds, st);
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
  double* part;
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

__global__ void k_field_setup(FieldWs w, int64_t n, int tiles_per_split_blocks, int S) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    ClusterParams cp = {};
    cp.off = 0;
    cp.cap = n;
    *w.cp = cp;
    ClusterDyn d = {};
    d.n_cur = n;
    d.i_blocks = tiles_per_split_blocks;
    d.n_tiles = tiles_per_split_blocks * S;
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

}  // namespace

int force_tile_targets(const ForceTiling& ft) { return (4 / ft.WJ) * 64 * ft.R; }

bool force_tiling_valid(int precision, const ForceTiling& ft) {
  bool r_ok = ft.R == 1 || ft.R == 2 || ft.R == 4 || (ft.R == 8 && precision != LC_FP64 && ft.WJ == 1);
  bool wj_ok = ft.WJ == 1 || ft.WJ == 2 || ft.WJ == 4;
  bool t_ok = ft.T >= 64 && ft.T <= 4096 && (ft.T % 64) == 0;
  if (ft.scalar_src && precision == LC_FP64) return false;  // scalar source path is FP32 only
  bool s_ok = ft.S >= 1 && ft.S <= 64;
  if (!(r_ok && wj_ok && t_ok && s_ok)) return false;
  return force_lds_bytes(precision, ft, true) <= 64 * 1024;
}

hipError_t launch_force(const DevState& s, const RunConst& rc, int precision, const ForceTiling& ft,
                        bool want_phi, int grid_blocks, hipStream_t st) {
  TileMap map{s.tile_start, s.order, s.cp, s.dyn, s.tile_total, s.queue, rc.n_clusters};
  const void* src = (precision == LC_FP64) ? (const void*)s.posq : (const void*)s.pos4;
  return launch_generic(precision, ft, map, src, s.part, rc.n_total, rc.eps2, want_phi, grid_blocks, st);
}

size_t field_workspace_bytes(int precision, int64_t n, const ForceTiling& ft) {
  size_t b = align256(sizeof(ClusterParams)) + align256(sizeof(ClusterDyn)) + 256;
  b += align256((size_t)n * (precision == LC_FP64 ? sizeof(double4) : sizeof(float4)));
  b += align256((size_t)ft.S * kComp * (size_t)n * sizeof(double));
  return b;
}

hipError_t launch_field_standalone(int precision, int64_t n, const double* xyzq, double eps2, double* E,
                                   double* phi, void* work, const ForceTiling& ft, hipStream_t st) {
  if (n == 0) return hipSuccess;
  FieldWs w = carve_field_ws(work, precision, n, ft);
  const int TI = force_tile_targets(ft);
  const int ib = (int)((n + TI - 1) / TI);
  k_field_setup<<<1, 64, 0, st>>>(w, n, ib, ft.S);
  const int pb = (int)((n + kBlock - 1) / kBlock);
  if (precision == LC_FP64) k_pack_sources<double4><<<pb, kBlock, 0, st>>>(xyzq, n, (double4*)w.src);
  else k_pack_sources<float4><<<pb, kBlock, 0, st>>>(xyzq, n, (float4*)w.src);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  TileMap map{w.ints, w.ints + 2, w.cp, w.dyn, w.ints + 3, w.ints + 4, 1};
  int grid = ib * ft.S;
  if (ft.persistent) {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int pg = cus * 8;
    grid = grid < pg ? grid : pg;
  }
  e = launch_generic(precision, ft, map, w.src, w.part, n, eps2, phi != nullptr, grid, st);
  if (e != hipSuccess) return e;
  k_sum_partials<<<pb, kBlock, 0, st>>>(w.part, n, ft.S, E, phi);
  return hipGetLastError();
}

}  // namespace lc

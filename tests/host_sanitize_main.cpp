// Host-side paths of the C ABI that need no GPU, for a build with AddressSanitizer and
// UndefinedBehaviorSanitizer: version and error strings, the pair-once row check over every
// shape and a range of capacities, the unit conversions, state sizing of valid and invalid
// configurations, and lc_create's argument validation (which rejects before any device work).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../include/lcmd.h"

static lc_config base_config(int precision) {
  lc_config c;
  std::memset(&c, 0, sizeof c);
  c.struct_size = sizeof(lc_config);
  c.precision = precision;
  c.ionize = 1;
  c.lambda_um = 0.8;
  c.dt = 0.05;
  c.softening_nm = 0.1;
  c.diag_every = 10;
  c.max_records = 64;
  c.max_splits = 8;
  c.max_pair_blocks = 64;
  c.seed = 1;
  c.detector_half_angle_deg = 30.0;
  c.box_r0 = 20.0;
  c.t_switch = INFINITY;
  return c;
}

static lc_cluster argon(int64_t n_ion, int64_t capacity) {
  lc_cluster k;
  std::memset(&k, 0, sizeof k);
  k.r0_nm = 2.5;
  k.rw_angstrom = 2.4;
  k.mass_u = 39.948;
  const double ip[] = {15.76, 27.63, 40.74, 59.58, 74.84, 91.29, 124.41, 143.46, 422.45};
  for (int z = 0; z < 9 && z < LC_MAX_Z; ++z) k.ip_ev[z] = ip[z];
  k.intensity_wcm2 = 1e16;
  k.envelope = LC_SIN2;
  k.n_cycles = 10.0;
  k.n_ion = n_ion;
  k.capacity = capacity;
  k.z_max = 8;
  k.electron_offset_nm = 0.01;
  return k;
}

int main() {
  int bad = 0;
  std::printf("version %d\n", lc_version());
  for (int code = -8; code <= 1; ++code)
    if (!lc_error_string(code)) ++bad;
  int64_t out[3];
  long fits = 0;
  for (int prec = 0; prec < 3; ++prec)
    for (int R = 0; R <= 8; ++R)
      for (int WJ = 0; WJ <= 6; ++WJ)
        for (int64_t cap = 1; cap <= 20000; cap += 97)
          if (lc_pair_rows_fit(prec, R, WJ, cap, 128, out) == LC_OK) ++fits;
  std::printf("row fits %ld\n", fits);
  if (fits == 0) ++bad;
  double u[6];
  if (lc_units(0.8, 1e16, u) != LC_OK || !(u[0] > 0.0)) ++bad;
  // state sizing: valid configurations of every precision and boundary, then invalid ones
  std::vector<lc_cluster> cl;
  for (int i = 0; i < 70; ++i) cl.push_back(argon(50 + 37 * i, 500 + 411 * i));
  for (int prec = 0; prec < 3; ++prec)
    for (int bnd = 0; bnd < 3; ++bnd)
      for (int ion = 0; ion < 2; ++ion) {
        lc_config c = base_config(prec);
        c.boundary = bnd;
        c.ionize = ion;
        if (prec == LC_FP32_KAHAN) c.max_pair_blocks = 0;
        if (bnd == LC_MIXED) c.t_switch = 10.0;
        const size_t b1 = lc_state_bytes(&c, cl.data(), 1);
        const size_t b70 = lc_state_bytes(&c, cl.data(), 70);
        const bool kahan_pbc = prec == LC_FP32_KAHAN && bnd != LC_OPEN;
        if (kahan_pbc ? (b1 != 0 || b70 != 0) : (b1 == 0 || b70 <= b1)) ++bad;
      }
  lc_config c = base_config(LC_FP32_ACC64);
  if (lc_state_bytes(nullptr, cl.data(), 1) != 0) ++bad;
  if (lc_state_bytes(&c, nullptr, 1) != 0) ++bad;
  if (lc_state_bytes(&c, cl.data(), 0) != 0) ++bad;
  lc_config wrong = c;
  wrong.struct_size = 4;
  if (lc_state_bytes(&wrong, cl.data(), 1) != 0) ++bad;
  wrong = c;
  wrong.dt = -1.0;
  if (lc_state_bytes(&wrong, cl.data(), 1) != 0) ++bad;
  lc_cluster k = argon(100, 50);  // capacity below the ion count
  if (lc_state_bytes(&c, &k, 1) != 0) ++bad;
  // lc_create rejects bad arguments before touching the device
  lc_sim* sim = nullptr;
  if (lc_create(&sim, &wrong, cl.data(), 1, nullptr, 0, nullptr) != LC_E_INVALID || sim) ++bad;
  if (lc_create(&sim, &c, &k, 1, nullptr, 0, nullptr) != LC_E_INVALID || sim) ++bad;
  if (lc_create(nullptr, &c, cl.data(), 1, nullptr, 0, nullptr) != LC_E_INVALID) ++bad;
  if (lc_create(&sim, &c, cl.data(), 1, nullptr, 16, nullptr) != LC_E_INVALID || sim) ++bad;
  lc_tuning t;
  std::memset(&t, 0, sizeof t);
  t.newton3 = 1;
  t.targets_per_lane = 4;
  t.waves_per_target = 4;
  for (int prec = 0; prec < 3; ++prec)
    for (int64_t n = 0; n < 70000; n += 6997) (void)lc_field_workspace_bytes(prec, n, n % 2 ? &t : nullptr);
  std::printf("bad %d\n", bad);
  return bad;
}

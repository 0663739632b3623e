/* Driver for the sanitizer build of the oracle (AddressSanitizer + UndefinedBehaviorSanitizer):
 * runs every entry point of lc_oracle.c on small inputs that reach all of its branches (initial
 * placement, open / periodic / mixed boundaries, linear and circular polarization, laser-only
 * and local ionization with spawns and capacity overflow, collisional ionization, detectors,
 * records) and exits 0.  Built and run by tests/test_oracle_sanitize.py; the oracle's source is
 * included so its static functions are instrumented too. */
#include "../oracle/lc_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double* dalloc(int64_t n) { return (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double)); }

static void one_run(int boundary, int pol, int ofi, int collisional, int64_t n_ion, int64_t cap, int64_t steps) {
  or_params p;
  memset(&p, 0, sizeof(p));
  p.dt = 0.05;
  p.eps2 = 7.854e-4 * 7.854e-4;
  p.kappa = 2.213205e-8;
  p.a0 = 0.3;
  p.envelope = OR_ENV_FLAT;
  p.phase = OR_PHASE_DIPOLE;
  p.weight = 5.0;
  p.mass_ion = 72820.75;
  p.ionize = 1;
  p.ofi_field = ofi;
  p.z_max = 8;
  p.diag_every = 3;
  double ip_ev[8] = {15.76, 27.63, 40.74, 59.58, 74.84, 91.29, 124.4, 143.5};
  for (int k = 0; k < 8; ++k) p.ip_au[k] = ip_ev[k] / 27.211386245988;
  p.field_au = 7.80477;
  p.rate_scale = 17.558;
  p.delta = 7.854e-5;
  p.n_atoms = 1130.28;
  p.mec2_ev = 510998.95;
  p.seed = 7;
  p.cluster = 2;
  p.n_ion = n_ion;
  p.polarization = pol;
  p.boundary = boundary;
  p.box = 0.03;
  p.t_switch = 0.5 * steps * p.dt;
  p.collisional = collisional;
  p.lotz_a = 4.5e-14;
  for (int k = 0; k < 8; ++k) { p.lotz_q[k] = 6.0 - k % 6; p.ci_ip_ev[k] = ip_ev[k]; }
  p.ci_r0 = 0.0196;
  p.ne_per_macro = 1e20;
  p.s_per_unit = 4.247e-16;
  double *x = dalloc(cap), *y = dalloc(cap), *z = dalloc(cap), *ux = dalloc(cap), *uy = dalloc(cap), *uz = dalloc(cap);
  double *wl = dalloc(cap), *wc = dalloc(cap), *wsp = dalloc(cap), *work = dalloc(8 * cap);
  int8_t* Z = (int8_t*)calloc((size_t)cap, 1);
  or_init(p.seed, p.cluster, n_ion, 1, p.ci_r0, p.delta, x, y, z, Z);
  int64_t n = 2 * n_ion;
  or_start(&p, n, x, y, z, ux, uy, uz, Z, work);
  or_detector det;
  or_detector_init(&det, 0.02, 30.0 * M_PI / 180.0);
  det.counts = (int64_t*)calloc(4 * OR_DET_SLOTS, sizeof(int64_t));
  det.seen = (int8_t*)calloc((size_t)cap, 1);
  double counters[2] = {0.0, 0.0};
  int64_t max_rec = steps / 3 + 2;
  double* rec = dalloc(max_rec * OR_REC);
  int64_t k = or_run(&p, cap, &n, x, y, z, ux, uy, uz, Z, wl, wc, wsp, 0, steps, work, counters, rec, max_rec, &det);
  double ex[5], ey[5], ez[5], phi[5];
  int64_t idx[5] = {0, n - 1, n / 2, 1, 0};
  or_coulomb_field_at(n, x, y, z, work, p.eps2, 5, idx, ex, ey, ez, phi);
  or_state_field(&p, 1.0, n, x, y, z, Z, work, work + cap, work + 2 * cap, work + 3 * cap, work + 4 * cap);
  printf("boundary %d pol %d ofi %d ci %d: n %lld records %lld events %.0f dropped %.0f\n", boundary, pol, ofi,
         collisional, (long long)n, (long long)k, counters[1], counters[0]);
  free(x); free(y); free(z); free(ux); free(uy); free(uz); free(wl); free(wc); free(wsp); free(work); free(Z);
  free(det.counts); free(det.seen); free(rec);
}

int main(void) {
  uint64_t key[2] = {1, 2}, ctr[4] = {3, 4, 5, 6}, out[4];
  or_philox4x64_10(key, ctr, out);
  double s = or_u01(out[0]) + or_adk_rate(0.5, 1.0, 0.05) + or_adk_rate(0.5, 1.0, 0.0) + or_e1(0.3) + or_e1(7.0) +
             or_lotz_rate(4.5e-14, 6.0, 15.76, 30.0) + or_lotz_rate(4.5e-14, 6.0, 15.76, 0.0);
  double E[3], B[3], uo[3] = {0.1, -0.2, 0.05}, un[3];
  or_params q;
  memset(&q, 0, sizeof(q));
  for (int env = 0; env < 4; ++env) {
    q.envelope = env; q.a0 = 0.1; q.tau = 70.0; q.t_sin2 = 60.0; q.phase = env & 1; q.polarization = env >> 1;
    or_laser(&q, 3.0, 0.01, E, B);
    s += or_envelope(&q, 100.0) + E[0] + B[1];
  }
  or_boris_push(-1.0, 0.05, E, B, uo, un);
  s += un[0];
  /* capacity 130 for 64 ions + 64 electrons: spawns beyond the second are dropped */
  one_run(OR_OPEN, OR_POL_LINEAR_X, OR_OFI_LASER_ONLY, 0, 64, 130, 30);
  one_run(OR_PERIODIC, OR_POL_CIRCULAR, OR_OFI_LOCAL, 1, 64, 1200, 30);
  one_run(OR_MIXED, OR_POL_LINEAR_X, OR_OFI_LOCAL, 1, 50, 900, 40);
  printf("checksum %.6e threads %d\n", s, or_threads());
  return 0;
}

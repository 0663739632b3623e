/*
 * lc_oracle.c -- plain FP64 CPU oracle for the laser-cluster molecular-dynamics step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call this
 * file; only the tests, the smoke check and the CPU-baseline leg of the benchmark do.
 * It shares no code, header, table or constant with the GPU library: every constant it
 * needs arrives through or_params (computed by oracle/units.py) or is written out here.
 *
 * Everything is in the paper's dimensionless units (Sec. II): fields in a0 = eE/(m_e w c)
 * and b0 = eB/(m_e w), time in 1/w, length in 1/k = c/w, momentum u = gamma*v/c, energy
 * in m_e c^2.  Arithmetic is IEEE FP64, built with -ffp-contract=off and without
 * fast-math; the only parallelism is OpenMP over the target index of the field sum,
 * which does not change any result.
 *
 * Pieces, in the order one time step uses them:
 *   or_coulomb_field  - direct sum over all other charges (Sec. II, force on each particle
 *                       from every other charged particle), Plummer-softened.
 *   or_laser          - dipole-approximation laser E/B with the Gaussian envelope of Eq.(3)
 *                       and the field components of Eqs.(4)-(9) (linear polarization).
 *   or_boris_push     - relativistic Boris leap-frog (Sec. II, Boris mover).
 *   or_adk_rate       - ADK tunnelling rate (cited in Sec. II; standard l = m = 0 form).
 *   ionization        - Monte-Carlo test P = 1 - exp(-nu dt) against alpha in (0,1]
 *                       (Sec. II), electron spawned next to the ion.
 *   or_lotz_rate      - collisional ionization rate (Sec. II: nu_total = nu_ofi + nu_ci), Lotz
 *                       form with the electron density and temperature of the cluster sphere.
 *   or_e1             - exponential integral E1 (series and continued fraction).
 *   or_sep,           - periodic, open or mixed boundaries of the simulation box (Sec. II):
 *   or_wrap             minimum-image separations and re-entry through the opposite face.
 *   or_detect         - ion detectors and the time-integrated ion energy distribution
 *                       (Sec. III anisotropy study: detectors at 9 R0, 30 degree acceptance).
 *   or_philox4x64_10  - Philox4x64-10 counter-based generator (Salmon et al., SC'11).
 *   or_init           - random placement of the ions inside R0 and of their electrons (Sec. II).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <string.h>

/* ---------------------------------------------------------------- Philox4x64-10 */
/* Multipliers and Weyl increments from Salmon, Moraes, Dror, Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3" (SC'11), Philox4x64. */
#define OR_PHILOX_M0 0xD2E7470EE14C6C93ULL
#define OR_PHILOX_M1 0xCA5A826395121157ULL
#define OR_PHILOX_W0 0x9E3779B97F4A7C15ULL
#define OR_PHILOX_W1 0xBB67AE8584CAA73BULL

static void or_mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
  unsigned __int128 p = (unsigned __int128)a * (unsigned __int128)b;
  *hi = (uint64_t)(p >> 64);
  *lo = (uint64_t)p;
}

/* Ten rounds; the key is bumped by the Weyl constants between rounds. */
void or_philox4x64_10(const uint64_t key_in[2], const uint64_t ctr_in[4], uint64_t out[4]) {
  uint64_t k0 = key_in[0], k1 = key_in[1];
  uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += OR_PHILOX_W0; k1 += OR_PHILOX_W1; }
    uint64_t hi0, lo0, hi1, lo1;
    or_mulhilo64(OR_PHILOX_M0, c0, &hi0, &lo0);
    or_mulhilo64(OR_PHILOX_M1, c2, &hi1, &lo1);
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    uint64_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform draw in (0, 1]: the top 53 bits plus one, times 2^-53.  The paper draws
 * 0 < alpha <= 1 (Sec. II, Monte-Carlo ionization). */
double or_u01(uint64_t x) { return (double)((x >> 11) + 1ULL) * (1.0 / 9007199254740992.0); }

/* ------------------------------------------------------------------ parameters */
enum { OR_ENV_GAUSS_FIELD = 0, OR_ENV_GAUSS_INTENSITY = 1, OR_ENV_SIN2 = 2, OR_ENV_FLAT = 3 };
enum { OR_PHASE_DIPOLE = 0, OR_PHASE_PLANE_WAVE = 1 };
enum { OR_POL_LINEAR_X = 0, OR_POL_CIRCULAR = 1 };
enum { OR_OPEN = 0, OR_PERIODIC = 1, OR_MIXED = 2 };
enum { OR_OFI_LASER_ONLY = 0, OR_OFI_LOCAL = 1 };
enum { OR_PURPOSE_ALPHA = 2, OR_PURPOSE_DIRECTION = 3 };

#define OR_MAX_Z 16
#define OR_REC 48 /* doubles per diagnostic record */

typedef struct {
  double dt, t0;        /* time step and start time (1/w)                          */
  double eps2;          /* Plummer softening squared ((c/w)^2)                     */
  double kappa;         /* Coulomb coupling r_e k: field of charge Q at r is kappa Q/r^2 */
  double a0;            /* peak field amplitude (a0 = b0)                          */
  int32_t envelope;     /* OR_ENV_*                                                */
  int32_t phase;        /* OR_PHASE_*                                              */
  double tau;           /* FWHM for the Gaussian envelopes (1/w)                   */
  double t_sin2;        /* total length T of the sin^2 envelope (1/w)              */
  double weight;        /* real particles per macroparticle                        */
  double mass_ion;      /* ion mass in m_e                                         */
  int32_t ionize;       /* 0: charges frozen                                       */
  int32_t ofi_field;    /* OR_OFI_*                                                */
  int32_t z_max;        /* highest ion charge reachable                            */
  int32_t diag_every;   /* diagnostic record every k steps (0: never)              */
  double ip_au[OR_MAX_Z]; /* ionization potential of Z -> Z+1 in Hartree, index Z  */
  double field_au;      /* atomic units of field per a0                            */
  double rate_scale;    /* (rate in 1/w) per (rate in atomic units)                */
  double delta;         /* distance of a spawned electron from its ion (c/w)       */
  double n_atoms;       /* real atoms in the cluster (Eq.(1), unrounded)           */
  double mec2_ev;       /* m_e c^2 in eV                                           */
  uint64_t seed;        /* Philox key word 0                                       */
  uint64_t cluster;     /* Philox key word 1                                       */
  int64_t n_ion;        /* ions occupy indices [0, n_ion)                          */
  int32_t polarization; /* OR_POL_*                                                */
  int32_t boundary;     /* OR_OPEN, OR_PERIODIC, or OR_MIXED (periodic while t < t_switch) */
  double box;           /* side L of the periodic cube centred on the cluster (c/w)  */
  double t_switch;      /* OR_MIXED: first time (1/w) with open boundaries             */
  int32_t collisional;  /* 1: add the collisional ionization rate to the ADK rate      */
  double lotz_a;        /* Lotz constant a (cm^2 eV^2)                                 */
  double lotz_q[OR_MAX_Z];  /* electrons in the outermost subshell of charge state Z  */
  double ci_ip_ev[OR_MAX_Z]; /* ionization energy Z -> Z+1 (eV)                      */
  double ci_r0;         /* radius of the sphere the electron density and temperature are
                           taken over, and inside which ions see them (c/w)            */
  double ne_per_macro;  /* real electrons per cm^3 that one macro-electron in it adds    */
  double s_per_unit;    /* seconds per unit of time (1/w)                               */
} or_params;

/* ------------------------------------------------------------------ boundaries */
/* Sec. II: periodic boundaries on the faces of a cube of side R_IC = 20 R0 around the cluster
 * stand in for the neighbouring clusters; open boundaries, or periodic ones first and open
 * ones afterwards (mixed), are the other options.  Periodic here means the minimum-image
 * convention: a pair interacts through the nearest periodic copy of the partner, and a
 * particle leaving the cube re-enters through the opposite face. */
/* Separation xi - xj through the nearest periodic copy (L > 0): d - L round(d / L), so a
 * separation inside (-L/2, L/2) is unchanged.  Which copy is nearest is an integer decided in
 * FP64 here; at an exact tie of L/2 the rounding (half to even) keeps d. */
static double or_sep(double xi, double xj, double L) {
  double d = xi - xj;
  if (!(L > 0.0)) return d;
  return d - L * nearbyint(d / L);
}

static double or_wrap(double x, double L) { return x - L * floor(x / L + 0.5); }

/* Side of the periodic cube in force at time t, or 0 when the boundaries are open. */
static double or_box_at(const or_params* p, double t) {
  if (p->boundary == OR_PERIODIC || (p->boundary == OR_MIXED && t < p->t_switch)) return p->box;
  return 0.0;
}

/* ------------------------------------------------------------------ S2: field */
/* E_i = sum_{j != i} q_j (r_i - r_j) / (|r_i - r_j|^2 + eps^2)^{3/2}
 * phi_i = sum_{j != i} q_j / (|r_i - r_j|^2 + eps^2)^{1/2}
 * q_j is the source strength in field units (kappa * weight * Z_j).  The j loop runs in
 * ascending order for every i.  L > 0: separations by the minimum-image convention in a
 * periodic cube of side L. */
static void or_field_one(int64_t i, int64_t n, const double* x, const double* y, const double* z,
                         const double* q, double eps2, double L, double out[4]) {
  double sx = 0.0, sy = 0.0, sz = 0.0, sp = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double dx = or_sep(x[i], x[j], L);
    double dy = or_sep(y[i], y[j], L);
    double dz = or_sep(z[i], z[j], L);
    double r2 = dx * dx + dy * dy + dz * dz + eps2;
    double inv = 1.0 / sqrt(r2);
    double inv3 = inv * inv * inv;
    double s = q[j] * inv3;
    sx += s * dx;
    sy += s * dy;
    sz += s * dz;
    sp += q[j] * inv;
  }
  out[0] = sx;
  out[1] = sy;
  out[2] = sz;
  out[3] = sp;
}

void or_coulomb_field_box(int64_t n, const double* x, const double* y, const double* z, const double* q,
                          double eps2, double L, double* ex, double* ey, double* ez, double* phi) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double o[4];
    or_field_one(i, n, x, y, z, q, eps2, L, o);
    ex[i] = o[0];
    ey[i] = o[1];
    ez[i] = o[2];
    if (phi) phi[i] = o[3];
  }
}

void or_coulomb_field(int64_t n, const double* x, const double* y, const double* z, const double* q,
                      double eps2, double* ex, double* ey, double* ez, double* phi) {
  or_coulomb_field_box(n, x, y, z, q, eps2, 0.0, ex, ey, ez, phi);
}

/* The same sum evaluated only at the m targets listed in idx (for sampled checks of large
 * states, open boundaries); outputs are indexed by position in idx. */
void or_coulomb_field_at(int64_t n, const double* x, const double* y, const double* z, const double* q,
                         double eps2, int64_t m, const int64_t* idx, double* ex, double* ey, double* ez,
                         double* phi) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    double o[4];
    or_field_one(idx[k], n, x, y, z, q, eps2, 0.0, o);
    ex[k] = o[0];
    ey[k] = o[1];
    ez[k] = o[2];
    if (phi) phi[k] = o[3];
  }
}

/* ------------------------------------------------------------------ S1: laser */
/* Envelope of the field amplitude.  Eq.(3) multiplies a0 by exp[-2.77 (t - 2 tau)^2/tau^2]
 * with the pulse centred at 2 tau; the constant is used as printed.  The intensity-FWHM
 * variant halves the exponent.  sin^2 and flat envelopes serve the test workloads. */
double or_envelope(const or_params* p, double t) {
  switch (p->envelope) {
    case OR_ENV_GAUSS_FIELD: {
      double d = t - 2.0 * p->tau;
      return p->a0 * exp(-2.77 * d * d / (p->tau * p->tau));
    }
    case OR_ENV_GAUSS_INTENSITY: {
      double d = t - 2.0 * p->tau;
      return p->a0 * exp(-1.385 * d * d / (p->tau * p->tau));
    }
    case OR_ENV_SIN2: {
      if (t <= 0.0 || t >= p->t_sin2) return 0.0;
      double s = sin(M_PI * t / p->t_sin2);
      return p->a0 * s * s;
    }
    default:
      return p->a0;
  }
}

/* Eqs.(4)-(9): E = a(t) (sin psi, sin(psi + phi_E), 0), B = a(t) (sin(psi + phi_B), sin psi, 0)
 * with b0 = a0 in these units.  Linear polarization along x takes the phases that make E_y
 * and B_x vanish.  Circular polarization takes phi_E = 3 pi/2 and phi_B = pi/2, so that
 * E_y = -a cos psi and B_x = a cos psi (each component with the full amplitude a(t)).
 * psi = t in the dipole approximation (the cluster is much smaller than the wavelength);
 * psi = t - z for the plane-wave test mode. */
void or_laser(const or_params* p, double t, double z, double E[3], double B[3]) {
  double psi = (p->phase == OR_PHASE_PLANE_WAVE) ? (t - z) : t;
  double env = or_envelope(p, t);
  double a = env * sin(psi);
  E[0] = a; E[1] = 0.0; E[2] = 0.0;
  B[0] = 0.0; B[1] = a; B[2] = 0.0;
  if (p->polarization == OR_POL_CIRCULAR) {
    double c = env * cos(psi);
    E[1] = -c;
    B[0] = c;
  }
}

/* ------------------------------------------------------------------ S3: Boris */
/* Relativistic Boris step for one macroparticle with charge-to-mass ratio zm = Z/M:
 * half electric kick, magnetic rotation, half electric kick. */
static void or_boris(double zm, double dt, const double E[3], const double B[3], const double uo[3],
                     double un[3]) {
  double h = 0.5 * zm * dt;
  double um[3] = {uo[0] + h * E[0], uo[1] + h * E[1], uo[2] + h * E[2]};
  double gm = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
  double tv[3] = {h * B[0] / gm, h * B[1] / gm, h * B[2] / gm};
  double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  double sv[3] = {2.0 * tv[0] / (1.0 + t2), 2.0 * tv[1] / (1.0 + t2), 2.0 * tv[2] / (1.0 + t2)};
  double up[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]),
                  um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                  um[2] + (um[0] * tv[1] - um[1] * tv[0])};
  double uplus[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]),
                     um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                     um[2] + (up[0] * sv[1] - up[1] * sv[0])};
  un[0] = uplus[0] + h * E[0];
  un[1] = uplus[1] + h * E[1];
  un[2] = uplus[2] + h * E[2];
}

/* Exposed for the single-particle tests. */
void or_boris_push(double zm, double dt, const double E[3], const double B[3], const double uo[3],
                   double un[3]) {
  or_boris(zm, dt, E, B, uo, un);
}

/* ------------------------------------------------------------------ S4: ADK */
/* Static ADK rate in atomic units for l = m = 0 with l* = n* - 1:
 *   n* = Zc / sqrt(2 Ip),  F0 = (2 Ip)^{3/2},  C^2 = 2^{2n*} / (n* Gamma(2 n*)),
 *   nu = C^2 Ip (2 F0 / F)^{2n* - 1} exp(-2 F0 / (3 F)),
 * evaluated in log space; nu = 0 below 1e-6 a.u. of field. */
double or_adk_rate(double ip, double zc, double f) {
  if (!(f >= 1e-6)) return 0.0;
  double ns = zc / sqrt(2.0 * ip);
  double f0 = pow(2.0 * ip, 1.5);
  double log_c2 = 2.0 * ns * log(2.0) - log(ns) - lgamma(2.0 * ns);
  double log_nu = log_c2 + log(ip) + (2.0 * ns - 1.0) * log(2.0 * f0 / f) - 2.0 * f0 / (3.0 * f);
  return exp(log_nu);
}

/* ------------------------------------------------------------------ collisional ionization */
/* Sec. II adds a collisional rate nu_ci to the tunnelling rate before the Monte-Carlo test.
 * The rate per ion is n_e <sigma v>, with the Lotz electron-impact cross-section of the
 * outermost subshell, sigma(E) = a q ln(E/P) / (E P) for E > P (q electrons bound by P), and a
 * Maxwellian electron energy distribution of temperature T:
 *   <sigma v> = int_P^inf sigma(E) sqrt(2E/m_e) 2 sqrt(E/pi) T^{-3/2} exp(-E/T) dE
 *             = 2 sqrt(2/(pi m_e)) a q E1(P/T) / (P sqrt(T))
 * (the logarithm integrated by parts).  n_e and T are taken over the electrons inside the
 * sphere of the initial cluster radius: n_e = (real electrons inside) / (sphere volume),
 * T = (2/3) x their mean kinetic energy; ions inside the sphere see them, ions outside none. */
#define OR_EV_J 1.602176634e-19
#define OR_ME_KG 9.1093837015e-31

/* E1(x), x > 0: power series E1 = -gamma - ln x - sum_k (-x)^k / (k k!) for x <= 1
 * (Abramowitz & Stegun 5.1.11), else the continued fraction of A&S 5.1.22 evaluated by the
 * modified Lentz method. */
double or_e1(double x) {
  if (x <= 1.0) {
    double sum = 0.0, term = 1.0;
    for (int k = 1; k < 100; ++k) {
      term *= -x / (double)k;
      double add = term / (double)k;
      sum += add;
      if (fabs(add) <= 1e-18 * fabs(sum)) break;
    }
    return -0.57721566490153286061 - log(x) - sum;
  }
  const double tiny = 1e-300;
  double b = x + 1.0, c = 1.0 / tiny, d = 1.0 / b, h = d;
  for (int i = 1; i < 1000; ++i) {
    double an = -(double)i * (double)i;
    b += 2.0;
    d = 1.0 / (an * d + b);
    c = b + an / c;
    double del = c * d;
    h *= del;
    if (fabs(del - 1.0) <= 1e-16) break;
  }
  return h * exp(-x);
}

/* <sigma v> (cm^3/s) for Lotz constant a (cm^2 eV^2), q outer electrons bound by P (eV), at
 * electron temperature T (eV); 0 without electrons or temperature. */
double or_lotz_rate(double a, double q, double P, double T) {
  if (!(T > 0.0) || !(q > 0.0) || !(P > 0.0)) return 0.0;
  double v1 = sqrt(2.0 * OR_EV_J / OR_ME_KG) * 100.0; /* sqrt(2 E / m_e) at E = 1 eV, cm/s */
  return 2.0 / sqrt(M_PI) * v1 * a * q * or_e1(P / T) / (P * sqrt(T));
}

/* ------------------------------------------------------------------ helpers */
static double or_mass(const or_params* p, int8_t Z) { return (Z < 0) ? 1.0 : p->mass_ion; }
static double or_gamma(double ux, double uy, double uz) { return sqrt(1.0 + ux * ux + uy * uy + uz * uz); }
/* gamma - 1 = u^2 / (1 + gamma), free of the cancellation of gamma - 1.0 for slow ions. */
static double or_gm1(double ux, double uy, double uz) {
  double u2 = ux * ux + uy * uy + uz * uz;
  return u2 / (1.0 + sqrt(1.0 + u2));
}

/* Source strengths for the field sum: kappa * w * Z. */
static void or_charges(const or_params* p, int64_t n, const int8_t* Z, double* q) {
  for (int64_t i = 0; i < n; ++i) q[i] = p->kappa * p->weight * (double)Z[i];
}

/* ------------------------------------------------------------------ initial placement */
/* Sec. II builds a cluster of radius R0 from atoms placed at random inside it and lumps them
 * into macroparticles (Eq.(1) gives the atom count; the weight is N_atoms / n_ion).  Each ion
 * starts with charge z_init and z_init electrons next to it.  Random numbers come from
 * Philox4x64-10 keyed by (seed, cluster):
 *   ion i (0 <= i < n_ion): counter (i, 0, 0, 0); its first three words give u1, u2, u3 in
 *     (0, 1] and the ion sits at radius R0 u1^{1/3} (uniform in volume) in the direction of
 *     polar cosine 2 u2 - 1 and azimuth 2 pi u3 (uniform on the sphere);
 *   electron e = i z_init + k of ion i (0 <= k < z_init): counter (e, 0, 1, 0); two words give
 *     the polar cosine and azimuth of its offset delta from the ion.
 * Order: the ions, then the electrons grouped by parent ion.  Momenta are zero.  x, y, z, Z
 * hold n_ion (1 + z_init) entries; positions in c/w. */
enum { OR_PURPOSE_ION = 0, OR_PURPOSE_ELECTRON = 1 };

static void or_direction(double u_cos, double u_phi, double d[3]) {
  double ct = 2.0 * u_cos - 1.0;
  double st = sqrt(fmax(0.0, 1.0 - ct * ct));
  double ph = 2.0 * M_PI * u_phi;
  d[0] = st * cos(ph);
  d[1] = st * sin(ph);
  d[2] = ct;
}

void or_init(uint64_t seed, uint64_t cluster, int64_t n_ion, int32_t z_init, double r0, double delta,
             double* x, double* y, double* z, int8_t* Z) {
  uint64_t key[2] = {seed, cluster};
  for (int64_t i = 0; i < n_ion; ++i) {
    uint64_t ctr[4] = {(uint64_t)i, 0, OR_PURPOSE_ION, 0};
    uint64_t r[4];
    or_philox4x64_10(key, ctr, r);
    double rad = r0 * cbrt(or_u01(r[0]));
    double d[3];
    or_direction(or_u01(r[1]), or_u01(r[2]), d);
    x[i] = rad * d[0];
    y[i] = rad * d[1];
    z[i] = rad * d[2];
    Z[i] = (int8_t)z_init;
  }
  for (int64_t i = 0; i < n_ion; ++i)
    for (int32_t k = 0; k < z_init; ++k) {
      int64_t e = i * z_init + k;
      uint64_t ctr[4] = {(uint64_t)e, 0, OR_PURPOSE_ELECTRON, 0};
      uint64_t r[4];
      or_philox4x64_10(key, ctr, r);
      double d[3];
      or_direction(or_u01(r[0]), or_u01(r[1]), d);
      x[n_ion + e] = x[i] + delta * d[0];
      y[n_ion + e] = y[i] + delta * d[1];
      z[n_ion + e] = z[i] + delta * d[2];
      Z[n_ion + e] = -1;
    }
}

/* ------------------------------------------------------------------ start */
/* Leap-frog start: one field pass at t0, then a backward half kick with the full
 * Lorentz force, u^{-1/2} = u^0 - (Z/M)(dt/2)(E + v^0 x B).  Returns sum w M (gamma - 1)
 * at the half step, the reference for the discrete energy identity.  work: 3*n doubles. */
double or_start(const or_params* p, int64_t n, const double* x, const double* y, const double* z,
                double* ux, double* uy, double* uz, const int8_t* Z, double* work) {
  double* q = work;
  double* ex = work + n;
  double* ey = work + 2 * n;
  double* ez = work + 3 * n;
  or_charges(p, n, Z, q);
  or_coulomb_field_box(n, x, y, z, q, p->eps2, or_box_at(p, p->t0), ex, ey, ez, NULL);
  double ke = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double EL[3], BL[3];
    or_laser(p, p->t0, z[i], EL, BL);
    double M = or_mass(p, Z[i]);
    if (Z[i] != 0) {
      double h = 0.5 * ((double)Z[i] / M) * p->dt;
      double g = or_gamma(ux[i], uy[i], uz[i]);
      double vx = ux[i] / g, vy = uy[i] / g, vz = uz[i] / g;
      double Ex = ex[i] + EL[0], Ey = ey[i] + EL[1], Ez = ez[i] + EL[2];
      double fx = Ex + (vy * BL[2] - vz * BL[1]);
      double fy = Ey + (vz * BL[0] - vx * BL[2]);
      double fz = Ez + (vx * BL[1] - vy * BL[0]);
      ux[i] -= h * fx;
      uy[i] -= h * fy;
      uz[i] -= h * fz;
    }
    ke += p->weight * M * or_gm1(ux[i], uy[i], uz[i]);
  }
  return ke;
}

/* ------------------------------------------------------------------ one step */
/* Diagnostic record layout (doubles):
 *  0 t^n  1 n  2 N  3 N_ion  4 N_electron
 *  5 KE at n+1/2: sum w M (gamma^{n+1/2} - 1)
 *  6 KE at n: sum w M ((gamma^{n-1/2} + gamma^{n+1/2})/2 - 1)
 *    (gamma - 1 is always evaluated as u^2 / (1 + gamma))
 *  7 PE at n: (1/2) sum_i w Z_i phi_i
 *  8 cumulative laser work W_L  9 cumulative Coulomb work W_C  10 cumulative spawn KE
 *  11-13 momentum sum w M u^{n+1/2}
 *  14-16 Coulomb force sum w Z E_C (Newton's third law makes this vanish)
 *  17 sum w |Z| |E_C| (scale for the residual above)
 *  18 mean ion charge  19 absorbed energy per atom in eV (W_L m_e c^2 / N_atoms)
 *  20 dropped spawns (cumulative)  21 ionization events (cumulative)
 *  22 laser envelope a(t^n)
 *  24.. 24+OR_MAX_Z: macro-ion count with charge Z = 0..OR_MAX_Z
 * The record describes the state after the push of step n and before its ionization. */

typedef struct {
  double* q;
  double* ex;
  double* ey;
  double* ez;
  double* phi;
  double* kebar;
  double* elx; /* laser field used at each particle this step (for OFI): x component */
  double* ely; /* and y component */
} or_scratch;

static void or_record(const or_params* p, int64_t step, int64_t n, const double* ux, const double* uy,
                      const double* uz, const int8_t* Z, const double* wl, const double* wc,
                      const double* wsp, const or_scratch* s, double dropped, double events,
                      double* rec) {
  memset(rec, 0, sizeof(double) * OR_REC);
  double t = p->t0 + (double)step * p->dt;
  rec[0] = t;
  rec[1] = (double)step;
  rec[2] = (double)n;
  double nion = 0.0, nel = 0.0, zsum = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double M = or_mass(p, Z[i]);
    double w = p->weight;
    rec[5] += w * M * or_gm1(ux[i], uy[i], uz[i]);
    rec[6] += s->kebar[i];
    rec[7] += 0.5 * w * (double)Z[i] * s->phi[i];
    rec[8] += wl[i];
    rec[9] += wc[i];
    rec[10] += wsp[i];
    rec[11] += w * M * ux[i];
    rec[12] += w * M * uy[i];
    rec[13] += w * M * uz[i];
    rec[14] += w * (double)Z[i] * s->ex[i];
    rec[15] += w * (double)Z[i] * s->ey[i];
    rec[16] += w * (double)Z[i] * s->ez[i];
    rec[17] += w * fabs((double)Z[i]) *
               sqrt(s->ex[i] * s->ex[i] + s->ey[i] * s->ey[i] + s->ez[i] * s->ez[i]);
    if (Z[i] < 0) {
      nel += 1.0;
    } else {
      nion += 1.0;
      zsum += (double)Z[i];
      if (Z[i] <= OR_MAX_Z) rec[24 + Z[i]] += 1.0;
    }
  }
  rec[3] = nion;
  rec[4] = nel;
  rec[18] = nion > 0.0 ? zsum / nion : 0.0;
  rec[19] = rec[8] * p->mec2_ev / p->n_atoms;
  rec[20] = dropped;
  rec[21] = events;
  rec[22] = or_envelope(p, t);
}

/* ------------------------------------------------------------------ detectors */
/* Ion detectors of the paper's anisotropy study (Sec. III): detectors at a distance D from
 * the cluster centre on the +-x (laser polarization), +-y and +-z axes; an ion is counted
 * once, at the first step its distance from the centre reaches D, by the detectors of every
 * axis whose direction its position vector makes an angle below the acceptance half-angle
 * with.  The time-integrated ion energy distribution is the histogram of the kinetic energy
 * of one real ion, M (gamma - 1) m_e c^2 in eV, at that step: 20 log-spaced bins per decade
 * from 1 eV to 1 MeV plus an underflow and an overflow bin, counted in macro-ions. */
#define OR_DET_BINS 120
#define OR_DET_SLOTS (OR_DET_BINS + 2)

typedef struct {
  double r2;                      /* D^2 ((c/w)^2)                                   */
  double cos2;                    /* cos^2 of the acceptance half-angle              */
  double edges[OR_DET_BINS + 1];  /* bin edges in eV                                 */
  int64_t* counts;                /* [4][OR_DET_SLOTS]: every ion, then the x, y, z axes */
  int8_t* seen;                   /* per index: 1 once counted                       */
} or_detector;

void or_detector_init(or_detector* d, double dist, double half_angle) {
  d->r2 = dist * dist;
  double c = cos(half_angle);
  d->cos2 = c * c;
  for (int k = 0; k <= OR_DET_BINS; ++k) d->edges[k] = pow(10.0, (double)k / 20.0);
}

/* Slot of energy e: the number of edges not above it (0 underflow, OR_DET_BINS + 1 overflow). */
static int or_det_slot(const or_detector* d, double e) {
  int k = 0;
  while (k <= OR_DET_BINS && d->edges[k] <= e) ++k;
  return k;
}

static void or_detect(const or_params* p, const or_detector* d, const double* x, const double* y,
                      const double* z, const double* ux, const double* uy, const double* uz,
                      const int8_t* Z) {
  for (int64_t i = 0; i < p->n_ion; ++i) {
    if (Z[i] <= 0 || d->seen[i]) continue;
    double r2 = x[i] * x[i] + y[i] * y[i] + z[i] * z[i];
    if (r2 < d->r2) continue;
    d->seen[i] = 1;
    double ev = or_mass(p, Z[i]) * or_gm1(ux[i], uy[i], uz[i]) * p->mec2_ev;
    int slot = or_det_slot(d, ev);
    d->counts[slot] += 1;
    double c[3] = {x[i], y[i], z[i]};
    for (int a = 0; a < 3; ++a)
      if (c[a] * c[a] > d->cos2 * r2) d->counts[(a + 1) * OR_DET_SLOTS + slot] += 1;
  }
}

/* One time step n (absolute index).  Field at x^n, laser at t^n = t0 + n dt, Boris push to
 * u^{n+1/2}, x^{n+1}, work split W_L / W_C, optional record, then the ionization check of
 * every ion in ascending index.  Returns the number of records written (0 or 1). */
static int or_step(const or_params* p, int64_t step, int64_t cap, int64_t* n_io, double* x, double* y,
                   double* z, double* ux, double* uy, double* uz, int8_t* Z, double* wl, double* wc,
                   double* wsp, const or_scratch* s, double* dropped, double* events, double* rec,
                   const or_detector* det) {
  int64_t n = *n_io;
  double t = p->t0 + (double)step * p->dt;
  int diag = (p->diag_every > 0) && (step % p->diag_every == 0);
  double L = or_box_at(p, t);
  or_charges(p, n, Z, s->q);
  or_coulomb_field_box(n, x, y, z, s->q, p->eps2, L, s->ex, s->ey, s->ez, s->phi);

#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double EL[3], BL[3];
    or_laser(p, t, z[i], EL, BL);
    s->elx[i] = EL[0];
    s->ely[i] = EL[1];
    double M = or_mass(p, Z[i]);
    double uo[3] = {ux[i], uy[i], uz[i]};
    double un[3] = {uo[0], uo[1], uo[2]};
    double go = or_gamma(uo[0], uo[1], uo[2]);
    if (Z[i] != 0) {
      double E[3] = {s->ex[i] + EL[0], s->ey[i] + EL[1], s->ez[i] + EL[2]};
      or_boris((double)Z[i] / M, p->dt, E, BL, uo, un);
    }
    double gn = or_gamma(un[0], un[1], un[2]);
    if (Z[i] != 0) {
      /* Exact discrete energy split: M (gamma_new - gamma_old) = Z dt E.(u_old+u_new)/(g_old+g_new),
       * linear in E, so the laser and Coulomb parts separate. */
      double c = p->weight * (double)Z[i] * p->dt / (go + gn);
      double sx = uo[0] + un[0], sy = uo[1] + un[1], sz = uo[2] + un[2];
      wl[i] += c * (EL[0] * sx + EL[1] * sy + EL[2] * sz);
      wc[i] += c * (s->ex[i] * sx + s->ey[i] * sy + s->ez[i] * sz);
    }
    s->kebar[i] = p->weight * M * 0.5 * (or_gm1(uo[0], uo[1], uo[2]) + or_gm1(un[0], un[1], un[2]));
    ux[i] = un[0];
    uy[i] = un[1];
    uz[i] = un[2];
    x[i] += p->dt * un[0] / gn;
    y[i] += p->dt * un[1] / gn;
    z[i] += p->dt * un[2] / gn;
    if (L > 0.0) {
      x[i] = or_wrap(x[i], L);
      y[i] = or_wrap(y[i], L);
      z[i] = or_wrap(z[i], L);
    }
  }

  if (det) or_detect(p, det, x, y, z, ux, uy, uz, Z);

  int wrote = 0;
  if (diag && rec) {
    or_record(p, step, n, ux, uy, uz, Z, wl, wc, wsp, s, *dropped, *events, rec);
    wrote = 1;
  }

  if (p->ionize) {
    uint64_t key[2] = {p->seed, p->cluster};
    double ne = 0.0, te = 0.0; /* electron density (cm^-3) and temperature (eV) in the sphere */
    double rr = p->ci_r0 * p->ci_r0;
    if (p->collisional) {
      double cnt = 0.0, ke = 0.0;
      for (int64_t j = 0; j < n; ++j) {
        if (Z[j] >= 0 || x[j] * x[j] + y[j] * y[j] + z[j] * z[j] >= rr) continue;
        cnt += 1.0;
        ke += or_gm1(ux[j], uy[j], uz[j]);
      }
      ne = cnt * p->ne_per_macro;
      te = (cnt > 0.0) ? (2.0 / 3.0) * (ke / cnt) * p->mec2_ev : 0.0;
    }
    int64_t n_base = n;
    for (int64_t i = 0; i < p->n_ion; ++i) {
      if (Z[i] < 0 || Z[i] >= p->z_max) continue;
      double ip = p->ip_au[Z[i]];
      if (!(ip > 0.0)) continue;
      double F;
      if (p->ofi_field == OR_OFI_LOCAL) {
        double fx = s->ex[i] + s->elx[i];
        double fy = s->ey[i] + s->ely[i];
        F = sqrt(fx * fx + fy * fy + s->ez[i] * s->ez[i]);
      } else if (p->polarization == OR_POL_CIRCULAR) {
        F = sqrt(s->elx[i] * s->elx[i] + s->ely[i] * s->ely[i]);
      } else {
        F = fabs(s->elx[i]);
      }
      double nu = or_adk_rate(ip, (double)Z[i] + 1.0, F * p->field_au) * p->rate_scale;
      if (p->collisional && x[i] * x[i] + y[i] * y[i] + z[i] * z[i] < rr)
        nu += ne * or_lotz_rate(p->lotz_a, p->lotz_q[Z[i]], p->ci_ip_ev[Z[i]], te) * p->s_per_unit;
      double P = -expm1(-nu * p->dt);
      uint64_t ctr[4] = {(uint64_t)i, (uint64_t)step, OR_PURPOSE_ALPHA, 0};
      uint64_t r[4];
      or_philox4x64_10(key, ctr, r);
      double alpha = or_u01(r[0]);
      if (!(alpha < P)) continue;
      if (n >= cap) {
        *dropped += 1.0;
        continue;
      }
      uint64_t ctr2[4] = {(uint64_t)i, (uint64_t)step, OR_PURPOSE_DIRECTION, 0};
      or_philox4x64_10(key, ctr2, r);
      double ct = 2.0 * or_u01(r[0]) - 1.0;
      double ph = 2.0 * M_PI * or_u01(r[1]);
      double st = sqrt(fmax(0.0, 1.0 - ct * ct));
      int64_t e = n++;
      x[e] = x[i] + p->delta * st * cos(ph);
      y[e] = y[i] + p->delta * st * sin(ph);
      z[e] = z[i] + p->delta * ct;
      if (L > 0.0) {
        x[e] = or_wrap(x[e], L);
        y[e] = or_wrap(y[e], L);
        z[e] = or_wrap(z[e], L);
      }
      ux[e] = ux[i];
      uy[e] = uy[i];
      uz[e] = uz[i];
      Z[e] = -1;
      wl[e] = 0.0;
      wc[e] = 0.0;
      wsp[e] = p->weight * or_gm1(ux[e], uy[e], uz[e]);
      Z[i] += 1;
      *events += 1.0;
    }
    (void)n_base;
  }
  *n_io = n;
  return wrote;
}

/* Run steps [step0, step0 + nsteps), counting detected ions in det unless it is NULL.  work
 * must hold 8*cap doubles.  Records go to rec
 * (OR_REC doubles each, at most max_rec); returns the number written.  counters[0] holds
 * dropped spawns and counters[1] ionization events, both carried across calls. */
int64_t or_run(const or_params* p, int64_t cap, int64_t* n_io, double* x, double* y, double* z,
               double* ux, double* uy, double* uz, int8_t* Z, double* wl, double* wc, double* wsp,
               int64_t step0, int64_t nsteps, double* work, double* counters, double* rec,
               int64_t max_rec, const or_detector* det) {
  or_scratch s;
  s.q = work;
  s.ex = work + cap;
  s.ey = work + 2 * cap;
  s.ez = work + 3 * cap;
  s.phi = work + 4 * cap;
  s.kebar = work + 5 * cap;
  s.elx = work + 6 * cap;
  s.ely = work + 7 * cap;
  int64_t nrec = 0;
  for (int64_t k = 0; k < nsteps; ++k) {
    double* r = (rec && nrec < max_rec) ? rec + nrec * OR_REC : NULL;
    nrec += or_step(p, step0 + k, cap, n_io, x, y, z, ux, uy, uz, Z, wl, wc, wsp, &s, &counters[0],
                    &counters[1], r, det);
  }
  return nrec;
}

/* Field of the current state only (the S2 step alone) at time t, for parity on a fixed state. */
void or_state_field(const or_params* p, double t, int64_t n, const double* x, const double* y, const double* z,
                    const int8_t* Z, double* q_work, double* ex, double* ey, double* ez, double* phi) {
  or_charges(p, n, Z, q_work);
  or_coulomb_field_box(n, x, y, z, q_work, p->eps2, or_box_at(p, t), ex, ey, ez, phi);
}

int or_record_size(void) { return OR_REC; }
int or_threads(void) { return omp_get_max_threads(); }
int or_max_z(void) { return OR_MAX_Z; }
int or_det_slots(void) { return OR_DET_SLOTS; }

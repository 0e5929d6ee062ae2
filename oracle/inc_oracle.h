/*
 * inc_oracle.h — C interface of the CPU oracle for the intranuclear-cascade +
 * evaporation method of Wan Chan Tseung & Beltran, "A graphics processor-based
 * intranuclear cascade and evaporation simulation" (arXiv:1309.7963).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, double-precision, scalar
 * implementation of the method, written from the paper (Sec. 2.1-2.4) and the
 * readings listed in the design notes.  Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load it.  It shares no code,
 * header, table or constant generator with the GPU library.
 *
 * Units: MeV, MeV/c, fm, mb.  Incident protons move along +z.
 */
#ifndef INC_ORACLE_H
#define INC_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NSHELL 15

/* Nuclear model of Sec. 2.2: 15 equal-thickness shells of a Fermi density. */
typedef struct {
  int A, Z;
  double c, delta, R;            /* Fermi parameters and outer radius (fm)   */
  double r[ORC_NSHELL + 1];      /* shell radii r_0 = 0 ... r_15 = R        */
  double integral[ORC_NSHELL];   /* int_{r_{i-1}}^{r_i} r^2 f(r) dr (fm^3)  */
  double rho[2][ORC_NSHELL];     /* [species n=0,p=1][shell] (fm^-3)        */
  double pF[2][ORC_NSHELL];      /* Fermi momenta (MeV/c)                   */
  double EF[2][ORC_NSHELL];      /* Fermi kinetic energies (MeV)            */
  double EB;                     /* binding energy per nucleon (MeV)        */
  double EC;                     /* Coulomb barrier e^2 Z / R (MeV)         */
} orc_nucleus;

/* Test hooks (all zero = the method as specified). */
typedef struct {
  int uniform_density;    /* every shell gets rho = A / (4/3 pi R^3)           */
  int zero_fermi;         /* pF = EF = 0 in every shell                       */
  int zero_binding;       /* EB = EC = 0                                      */
  int no_pauli;           /* skip the Pauli test                              */
  int no_evaporation;     /* stop after the cascade                           */
  int stop_after_first;   /* end the cascade at the first accepted collision  */
  double const_sigma_mb;  /* > 0: every NN cross-section is this constant     */
  double fixed_b;         /* >= 0: fixed impact parameter (fm); < 0: sampled  */
  int max_stack;          /* 0 = default 64                                   */
  int max_segments;       /* 0 = default 10000                                */
  int photon_evaporation; /* 1: photons compete with the particle channels of
                             the evaporation (reading R19; off by default)    */
  int heavy_fragments;    /* 1: the stable isotopes of Li to Mg are emitted
                             too, channels 7-26 (reading R20; off by default) */
} orc_options;

/* Per-event result.  Stage-0 (cascade) and stage-1 (evaporation) secondaries
 * are stored separately (see orc_run). */
typedef struct {
  int A_casc, Z_casc;     /* residual after the cascade                       */
  int A_f, Z_f;           /* residual after evaporation                       */
  double Ex_casc;         /* excitation after the cascade (MeV)               */
  double Ex_f;            /* excitation left after evaporation (MeV)          */
  double p_casc[3];       /* residual momentum after the cascade (MeV/c)      */
  double p_f[3];          /* final residual momentum (MeV/c)                  */
  int n_sec;              /* secondaries of this event                        */
  int flags;              /* 1 stack guard, 2 segment guard, 4 A'=0           */
  int n_retry;            /* transparent passes before the event              */
  int n_coll;             /* accepted (unblocked) NN collisions               */
  int n_tent;             /* tentative collisions                             */
  int n_pauli;            /* Pauli-blocked collisions                         */
  int n_seg;              /* flight segments                                  */
  int n_evap;             /* evaporation steps                                */
  int n_draw;             /* uniforms consumed                                */
  double first_z;         /* z of the first accepted collision (fm)           */
  int sea[2];             /* nucleons of each species (n, p) left in the Fermi
                             sea when the cascade ends                        */
  int sea_min;            /* lowest occupancy of either species reached      */
  uint32_t tent_shells;   /* h = 3 h + shell + 1 over the tentative collisions
                             in order, from h = 0 (mod 2^32): where they
                             happened, a fingerprint of the event's path      */
  int n_tau;              /* optical depths drawn, over all passes (each new
                             flight and each null or blocked collision)       */
  int n_majorant;         /* flight majorants evaluated (each new flight)     */
} orc_result;

typedef struct {
  uint32_t event;         /* event index within the batch                     */
  int species;            /* 0 n, 1 p, 2 d, 3 t, 4 3He, 5 alpha, 6 photon,
                             7-26 the heavier fragments (orc_fragment)        */
  int stage;              /* 0 cascade, 1 evaporation                         */
  double T;               /* kinetic energy (MeV)                             */
  double u[3];            /* direction (lab)                                  */
} orc_secondary;

/* --- building blocks, exposed for the pins ------------------------------ */
void   orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_uniform(uint32_t w);
/* k-th uniform (0-based) of the per-event stream of (seed, event id). */
double orc_stream_uniform(uint64_t seed, uint64_t event_id, uint64_t k);

double orc_binding(int A, int Z);     /* B(A,Z) (MeV)                          */
double orc_mass(int A, int Z);        /* nuclear mass (MeV)                    */
int    orc_nucleus_setup(int A, int Z, const orc_options* opt, orc_nucleus* out);

double orc_sigma(int like, double p_GeV);     /* NN elastic (mb)             */
double orc_sigma_hat(int like, double pmin_GeV); /* max of sigma over [pmin, top] */
double orc_slope(int like, double p_GeV);     /* b in (GeV/c)^-2             */
double orc_plab_min(double p, double mx, double pF, double my);

/* Elastic NN collision in the lab.  Inputs: projectile momentum px[3] (mass
 * mx), target momentum pt[3] (mass my), slope b, uniforms for the polar and
 * azimuthal CM angles.  Outputs: final momenta and kinetic energies.
 * Returns p_lab (MeV/c). */
double orc_elastic(const double px[3], double mx, const double pt[3], double my,
                   double b_GeV2, double u_theta, double u_phi,
                   double qx[3], double qt[3], double* Tx, double* Tt);

/* Refraction at a sphere (outward normal n).  T_in, T_out kinetic energies on
 * the two sides.  Returns 1 transmitted, 0 reflected; d is updated in place. */
int orc_refract(double d[3], const double n[3], double T_in, double T_out, double m);

/* Sec. 2.3 decision after an elastic collision in shell `shell` between a
 * moving nucleon of species sp_x and a target of species sp_y (0 n, 1 p):
 * product kinetic energies Tx, Ty, target kinetic energy Tt before it.
 * Returns bit 0 = Pauli-blocked (only when pauli != 0), bit 1 = the moving
 * product is tracked (else captured by the cutoff), bit 2 = the struck product
 * is tracked; out = {eps_x, eps_y, hole depth}.  -1 on bad arguments. */
int orc_collision_outcome(const orc_nucleus* nu, int shell, int sp_x, int sp_y, double Tx, double Ty, double Tt,
                          int pauli, double out[3]);

double orc_width_integral(double a, double U);   /* I(a,U) */
double orc_spectrum_cdf(double a, double U, double x);
double orc_spectrum_sample(double a, double U, double u);
/* photon channel (option, reading R19) */
double orc_gdr_energy(int A);                    /* E_G (MeV)                 */
double orc_photon_s0(int A, int Z);              /* sigma_g / eps (fm^2/MeV)  */
double orc_photon_integral(double a, double U);  /* J(a,U)                    */
double orc_photon_cdf(double a, double U, double x);
double orc_photon_sample(double a, double U, double u);
/* Emitted species j (0-5 particles, 7-26 heavier fragments; 6 the photon):
 * mass number, charge and ground-state spin multiplicity 2s + 1.  Returns 0
 * for j outside 0..26 or j = 6. */
int orc_fragment(int j, int* a, int* z, int* g);
double orc_photon_width(int A, int Z, double E); /* channel weight, 0 closed  */

/* Sample a target momentum uniform in a Fermi sphere of radius pF. */
void orc_fermi_sample(double pF, double u1, double u2, double u3, double p[3]);

/* Evaporation (Sec. 2.4) of an excited nucleus (A, Z, Ex, momentum P) with the
 * stream of (seed, event_id).  Of opt (NULL: defaults) only
 * photon_evaporation applies.  Fills res->A_f, Z_f, Ex_f, p_f, n_evap, n_draw
 * and up to sec_cap secondaries; returns the number emitted or -1. */
int orc_evaporate(int A, int Z, double Ex, const double P[3], uint64_t seed, uint64_t event_id,
                  const orc_options* opt, orc_result* res, orc_secondary* sec, int sec_cap);

/* --- event generation ----------------------------------------------------
 * targets: n_targets (A,Z) pairs.  tidx: per-event target index (NULL = 0).
 * T0: per-event incident kinetic energy (MeV).  Event i uses the stream of
 * (seed, first_id + i).  res: n entries.  sec: capacity sec_cap; the
 * secondaries are written in event order.  Returns the number of secondaries
 * (which may exceed sec_cap: then only sec_cap were stored), or -1 on an
 * argument error. */
int64_t orc_run(const int* targets_AZ, int n_targets, const orc_options* opt,
                size_t n, const uint8_t* tidx, const double* T0,
                uint64_t seed, uint64_t first_id,
                orc_result* res, orc_secondary* sec, size_t sec_cap,
                int n_threads);

#ifdef __cplusplus
}
#endif
#endif

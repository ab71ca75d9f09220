/*
 * lbmref.h -- FP64 CPU oracle for the variable-speed-of-sound D2Q9 lattice
 * Boltzmann model of Buick & Cosgrove, "Investigation of a Lattice Boltzmann
 * Model with a Variable Speed of Sound".
 *
 * TEST INFRASTRUCTURE. This library exists only so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check and time the GPU
 * library against a plain, slow, obviously correct implementation. The
 * product path (liblbm) never links, loads or calls it, and it shares no
 * source, header, table or helper with the product path.
 *
 * Model (paper Sec. 3, Eq. 5):
 *   f_i(x + e_i, t + 1) - f_i(x, t) = -(f_i - feq_i)/tau + 3 w_i alpha grad(rho).e_i
 * on a periodic nx x ny lattice, with the D2Q9 links and weights of Sec. 2,
 * the equilibrium of Eq. 2, the moments of Eq. 3, and the density gradient
 * taken by central differences (Sec. 4, discussion of Fig. 1).
 * The effective speed of sound is c_e^2 = 1/3 - alpha (Eq. 8); the library
 * is parameterised by c2 = c_e^2, so alpha = 1/3 - c2 and c2 = 1/3 is the
 * standard lattice Boltzmann model.
 *
 * Conventions: every field array is row-major with index y*nx + x; the
 * population array f has layout [9][ny][nx]. All arithmetic is IEEE FP64.
 */
#ifndef LBMREF_H
#define LBMREF_H

#ifdef __cplusplus
extern "C" {
#endif

enum lbmref_status {
    LBMREF_OK = 0,
    LBMREF_EINVAL = -1,     /* argument out of range                        */
    LBMREF_ENOMEM = -2,     /* host allocation failed                       */
    LBMREF_ESTATE = -4,     /* step or read before init                     */
    LBMREF_ENONFINITE = -5  /* a total is NaN or infinite                   */
};

typedef struct lbmref lbmref;

/* Lattice constants evaluated from the link-vector formulas of Sec. 2:
 * e[2*i+0], e[2*i+1] = (e_ix, e_iy); w[i] = weight. i = 0..8. */
void lbmref_lattice(int e[18], double w[9]);

/* alpha of Eq. 5 for a requested c_e^2 (Eq. 8 with c_1^2 = 1/3). */
double lbmref_alpha(double c2);

/* Eq. 2: feq[i] = w_i rho [1 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u]. */
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9]);

/* Source term of Eq. 5: s[i] = 3 w_i alpha (e_ix gx + e_iy gy). */
void lbmref_source(double alpha, double gx, double gy, double s[9]);

/* The other route to a free speed of sound that the paper discusses (Sec. 3,
 * opening): alter the equilibrium, i.e. the share of rest and moving
 * particles, instead of adding a force. On D2Q9 with sound speed c:
 *   feq[i] = w_i rho [3 c^2 + 3 e_i.u + 9/2 (e_i.u)^2 - 3/2 u.u]   (i != 0)
 *   feq[0] = rho - sum_{i != 0} feq[i]
 * whose moments are rho, rho u and c^2 rho I + rho u u; c^2 = 1/3 gives
 * Eq. 2. Used by LBMREF_MODEL_EQUILIBRIUM. */
void lbmref_equilibrium_c2(double c2, double rho, double ux, double uy, double feq[9]);

/* Which model a lattice steps (lbmref_set_model): the paper's Eq. 5
 * (default), or relaxation to lbmref_equilibrium_c2 with no source term. */
enum lbmref_model { LBMREF_MODEL_FORCING = 0, LBMREF_MODEL_EQUILIBRIUM = 1 };

/* Create a periodic nx x ny lattice. nx, ny >= 3; tau > 1/2 (Eq. 4 gives
 * nu > 0); c2 > 0 (Eq. 8). Returns NULL and sets lbmref_last_error() on
 * failure. */
lbmref* lbmref_create(int nx, int ny, double tau, double c2);
int lbmref_last_error(void);
void lbmref_destroy(lbmref* L);

/* Select the model (enum lbmref_model) before init; LBMREF_EINVAL for an
 * unknown model, for the equilibrium model with c2 >= 3/5 (its rest
 * population feq[0] = rho (1 - 5 c^2 / 3) would not be positive), or for the
 * equilibrium model on a lattice with a c2 field. */
int lbmref_set_model(lbmref* L, int model);

/* A speed of sound that varies in space (the paper's outlook, Sec. 5: alpha
 * need not be constant; e.g. an acoustic lens or a temperature gradient).
 * c2 has nx*ny entries, c2[y*nx + x] = c_e^2 at that site; the source term
 * of Eq. 5 at x then uses alpha(x) = 1/3 - c2[x] (Eq. 8 site by site), and
 * the gradient stays the central difference of rho. NULL restores the
 * lattice's uniform c2. May be called between steps (alpha varying in
 * time). LBMREF_EINVAL for a non-finite or non-positive entry, or for a
 * lattice on the equilibrium model (the field is a forcing-model feature);
 * the lattice keeps its previous field then. */
int lbmref_set_c2_field(lbmref* L, const double* c2);

/* Boundaries in x. LBMREF_XBC_PERIODIC (default): periodic, as everywhere
 * else. LBMREF_XBC_INLET_OUTLET: the set-up of Fig. 1 (Sec. 4), an
 * oscillating density at x = 0 and rho = 1, u = 0 at the far end. The
 * sites of columns x = 0 and x = nx - 1 do not collide: in the step from
 * time t they emit the model's equilibrium at rest, at the density
 * rho_in(t) = 1 + amplitude sin(2 pi t / period) (x = 0) and 1
 * (x = nx - 1). The periodic seam between the two columns is cut: a
 * population that would cross it (leaving x = 0 towards -x, or x = nx - 1
 * towards +x) arrives as the equilibrium population of the column it
 * enters, at that column's boundary density. y stays periodic.
 * LBMREF_EINVAL for an unknown mode, or for the inlet/outlet with nx < 5,
 * period not finite and > 0, or |amplitude| not < 1. */
enum lbmref_xbc { LBMREF_XBC_PERIODIC = 0, LBMREF_XBC_INLET_OUTLET = 1 };
int lbmref_set_x_boundaries(lbmref* L, int mode, double amplitude, double period);

/* f_i(x, 0) = feq_i(rho(x), u(x)) of the lattice's model. NULL rho means rho = 1, NULL ux / uy
 * mean 0. Arrays have nx*ny entries. Sets t = 0. */
int lbmref_init(lbmref* L, const double* rho, const double* ux, const double* uy);

/* Advance n >= 0 time steps of Eq. 5. */
int lbmref_step(lbmref* L, int n);

/* rho, u = j/rho of the current state (Eq. 3); any pointer may be NULL.
 * totals = {sum rho, sum j_x, sum j_y} (compensated FP64 sums in row-major
 * site order). Returns LBMREF_ENONFINITE if a total is not finite. */
int lbmref_moments(lbmref* L, double* rho, double* ux, double* uy, double totals[3]);

/* Canonical populations f_i(x, t), layout [9][ny][nx]. */
int lbmref_get_f(lbmref* L, double* f);
int lbmref_set_f(lbmref* L, const double* f);

/* Number of completed steps since init / set_f. */
long long lbmref_time(const lbmref* L);

/* OpenMP threads used by the site loops (n <= 0: library default).
 * Per-site arithmetic does not depend on the thread count. */
void lbmref_set_threads(int n);
int lbmref_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif /* LBMREF_H */

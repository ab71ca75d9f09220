/*
 * lbmref.c -- FP64 CPU oracle for the variable-speed-of-sound D2Q9 lattice
 * Boltzmann step. TEST INFRASTRUCTURE ONLY (see lbmref.h): used by tests,
 * the smoke check and the benchmark's CPU-baseline leg, never by the product
 * path, and sharing nothing with it.
 *
 * The code follows the paper's equations in order and in their notation;
 * it is written for reading, not for speed. Build: -O2 -ffp-contract=off,
 * no fast-math (see Makefile).
 */
#include "lbmref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct lbmref {
    int nx, ny;
    double tau;     /* relaxation time, Eq. 1                              */
    double alpha;   /* forcing amplitude, Eq. 5; alpha = 1/3 - c_e^2       */
    double c2;      /* c_e^2 as requested                                  */
    int model;      /* enum lbmref_model                                   */
    double* A;      /* alpha(x) of a c2 field, [ny][nx]; NULL: uniform     */
    int xbc;        /* enum lbmref_xbc                                     */
    double amp, period; /* inlet density oscillation (LBMREF_XBC_INLET_OUTLET) */
    long long t;    /* completed steps                                     */
    int ready;      /* set by init / set_f                                 */
    double* f;      /* f_i(x, t), [9][ny][nx]                              */
    double* fnew;   /* streaming target                                    */
    double* R;      /* rho(x, t), [ny][nx]                                 */
    double* UX;     /* u_x(x, t)                                           */
    double* UY;     /* u_y(x, t)                                           */
};

static _Thread_local int g_last_error = LBMREF_OK;

/* e_i and w_i, evaluated once by lbmref_lattice() when the library loads. */
static int E[18];
static double W[9];

int lbmref_last_error(void) { return g_last_error; }

/* ---------------------------------------------------------------------
 * Lattice (Sec. 2). Link vectors
 *   e_i = (cos[pi(i-1)/2], sin[pi(i-1)/2])               for i = 1..4,
 *   e_i = sqrt(2) (cos[pi(i-9/2)/2], sin[pi(i-9/2)/2])   for i = 5..8,
 *   e_0 = (0, 0);
 * weights w_0 = 4/9, w_1..4 = 1/9, w_5..8 = 1/36.
 * The components are integers; they are evaluated from the formulas and
 * rounded to the nearest integer.
 * ------------------------------------------------------------------- */
void lbmref_lattice(int e[18], double w[9])
{
    const double pi = 3.14159265358979323846;
    e[0] = 0;
    e[1] = 0;
    for (int i = 1; i <= 4; ++i) {
        double a = pi * (i - 1) / 2.0;
        e[2 * i + 0] = (int)lround(cos(a));
        e[2 * i + 1] = (int)lround(sin(a));
    }
    for (int i = 5; i <= 8; ++i) {
        double a = pi * (i - 4.5) / 2.0;
        e[2 * i + 0] = (int)lround(sqrt(2.0) * cos(a));
        e[2 * i + 1] = (int)lround(sqrt(2.0) * sin(a));
    }
    w[0] = 4.0 / 9.0;
    for (int i = 1; i <= 4; ++i) w[i] = 1.0 / 9.0;
    for (int i = 5; i <= 8; ++i) w[i] = 1.0 / 36.0;
}

__attribute__((constructor)) static void load_lattice(void) { lbmref_lattice(E, W); }

/* Eq. 8 with c_1^2 = 1/3: c_e^2 = 1/3 - alpha, so alpha = 1/3 - c_e^2.
 * (alpha = 1/3 gives c_e = 0 and alpha = -2/3 gives c_e = 1, Sec. 4.) */
double lbmref_alpha(double c2) { return 1.0 / 3.0 - c2; }

/* Eq. 2. */
void lbmref_equilibrium(double rho, double ux, double uy, double feq[9])
{
    const int* e = E;
    const double* w = W;
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double eu = e[2 * i] * ux + e[2 * i + 1] * uy;
        feq[i] = w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
    }
}

/* Extra term on the right-hand side of Eq. 5: 3 w_i alpha grad(rho).e_i,
 * with grad(rho) = (gx, gy). */
void lbmref_source(double alpha, double gx, double gy, double s[9])
{
    const int* e = E;
    const double* w = W;
    for (int i = 0; i < 9; ++i)
        s[i] = 3.0 * w[i] * alpha * (gx * e[2 * i] + gy * e[2 * i + 1]);
}

/* Altered equilibrium (the equilibrium route of Sec. 3 on D2Q9): the
 * moving populations carry 3 c^2 in place of the 1 of Eq. 2 and the rest
 * population takes what is left of rho. */
void lbmref_equilibrium_c2(double c2, double rho, double ux, double uy, double feq[9])
{
    const int* e = E;
    const double* w = W;
    double usq = ux * ux + uy * uy;
    double moving = 0.0;
    for (int i = 1; i < 9; ++i) {
        double eu = e[2 * i] * ux + e[2 * i + 1] * uy;
        feq[i] = w[i] * rho * (3.0 * c2 + 3.0 * eu + 4.5 * eu * eu - 1.5 * usq);
        moving += feq[i];
    }
    feq[0] = rho - moving;
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

int lbmref_set_model(lbmref* L, int model)
{
    if (!L) return LBMREF_EINVAL;
    if (model == LBMREF_MODEL_FORCING) {
        L->model = model;
        return LBMREF_OK;
    }
    if (model == LBMREF_MODEL_EQUILIBRIUM && L->c2 < 0.6 && !L->A) {
        L->model = model;
        return LBMREF_OK;
    }
    return LBMREF_EINVAL;
}

/* The equilibrium of the lattice's model. */
static void model_equilibrium(const lbmref* L, double rho, double ux, double uy, double feq[9])
{
    if (L->model == LBMREF_MODEL_EQUILIBRIUM) lbmref_equilibrium_c2(L->c2, rho, ux, uy, feq);
    else lbmref_equilibrium(rho, ux, uy, feq);
}

lbmref* lbmref_create(int nx, int ny, double tau, double c2)
{
    /* nx, ny >= 3 so the central differences of Sec. 4 see two distinct
     * neighbours; tau > 1/2 so nu = (2 tau - 1)/6 > 0 (Eq. 4); c2 > 0 so
     * c_e of Eq. 8 is real. */
    if (nx < 3 || ny < 3 || !isfinite(tau) || !(tau > 0.5) || !isfinite(c2) ||
        !(c2 > 0.0) || (long long)nx * ny > (1LL << 31) / 16) {
        g_last_error = LBMREF_EINVAL;
        return NULL;
    }
    lbmref* L = (lbmref*)calloc(1, sizeof(lbmref));
    if (!L) {
        g_last_error = LBMREF_ENOMEM;
        return NULL;
    }
    size_t n = (size_t)nx * ny;
    L->nx = nx;
    L->ny = ny;
    L->tau = tau;
    L->alpha = lbmref_alpha(c2);
    L->c2 = c2;
    L->model = LBMREF_MODEL_FORCING;
    L->f = (double*)calloc(9 * n, sizeof(double));
    L->fnew = (double*)calloc(9 * n, sizeof(double));
    L->R = (double*)calloc(n, sizeof(double));
    L->UX = (double*)calloc(n, sizeof(double));
    L->UY = (double*)calloc(n, sizeof(double));
    if (!L->f || !L->fnew || !L->R || !L->UX || !L->UY) {
        lbmref_destroy(L);
        g_last_error = LBMREF_ENOMEM;
        return NULL;
    }
    g_last_error = LBMREF_OK;
    return L;
}

void lbmref_destroy(lbmref* L)
{
    if (!L) return;
    free(L->f);
    free(L->fnew);
    free(L->R);
    free(L->UX);
    free(L->UY);
    free(L->A);
    free(L);
}

int lbmref_set_x_boundaries(lbmref* L, int mode, double amplitude, double period)
{
    if (!L) return LBMREF_EINVAL;
    if (mode == LBMREF_XBC_PERIODIC) {
        L->xbc = mode;
        return LBMREF_OK;
    }
    if (mode != LBMREF_XBC_INLET_OUTLET || L->nx < 5 || !isfinite(period) || !(period > 0.0) ||
        !isfinite(amplitude) || !(fabs(amplitude) < 1.0))
        return LBMREF_EINVAL;
    L->xbc = mode;
    L->amp = amplitude;
    L->period = period;
    return LBMREF_OK;
}

int lbmref_set_c2_field(lbmref* L, const double* c2)
{
    if (!L || L->model != LBMREF_MODEL_FORCING) return LBMREF_EINVAL;
    size_t n = (size_t)L->nx * L->ny;
    if (!c2) {
        free(L->A);
        L->A = NULL;
        return LBMREF_OK;
    }
    for (size_t s = 0; s < n; ++s)
        if (!isfinite(c2[s]) || !(c2[s] > 0.0)) return LBMREF_EINVAL;
    if (!L->A) {
        L->A = (double*)malloc(n * sizeof(double));
        if (!L->A) return LBMREF_ENOMEM;
    }
    /* Eq. 8 at every site */
    for (size_t s = 0; s < n; ++s) L->A[s] = lbmref_alpha(c2[s]);
    return LBMREF_OK;
}

int lbmref_init(lbmref* L, const double* rho, const double* ux, const double* uy)
{
    if (!L) return LBMREF_EINVAL;
    int nx = L->nx, ny = L->ny;
    size_t n = (size_t)nx * ny;
    for (size_t s = 0; s < n; ++s) {
        double feq[9];
        model_equilibrium(L, rho ? rho[s] : 1.0, ux ? ux[s] : 0.0, uy ? uy[s] : 0.0, feq);
        for (int i = 0; i < 9; ++i) L->f[i * n + s] = feq[i];
    }
    L->t = 0;
    L->ready = 1;
    return LBMREF_OK;
}

/* Eq. 3 at every site: rho = sum_i f_i, rho u = sum_i f_i e_i. */
static void compute_moments(lbmref* L)
{
    const int* e = E;
    int nx = L->nx, ny = L->ny;
    size_t n = (size_t)nx * ny;
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            double rho = 0.0, jx = 0.0, jy = 0.0;
            for (int i = 0; i < 9; ++i) {
                double fi = L->f[i * n + s];
                rho += fi;
                jx += fi * e[2 * i];
                jy += fi * e[2 * i + 1];
            }
            L->R[s] = rho;
            L->UX[s] = jx / rho;
            L->UY[s] = jy / rho;
        }
    }
}

/* One time step of Eq. 5 (or of the equilibrium model: relaxation to
 * lbmref_equilibrium_c2, no source term). */
static void step_once(lbmref* L)
{
    const int* e = E;
    int nx = L->nx, ny = L->ny;
    size_t n = (size_t)nx * ny;

    /* rho(x, t) and u(x, t) from Eq. 3. */
    compute_moments(L);

    /* Fig. 1 boundaries: what the two boundary columns emit in this step,
     * their equilibria at rest at the inlet density and at rho = 1. */
    const int xbc = L->xbc == LBMREF_XBC_INLET_OUTLET;
    double fin[9], fout[9];
    if (xbc) {
        const double pi = 3.14159265358979323846;
        double rho_in = 1.0 + L->amp * sin(2.0 * pi * (double)L->t / L->period);
        model_equilibrium(L, rho_in, 0.0, 0.0, fin);
        model_equilibrium(L, 1.0, 0.0, 0.0, fout);
    }

#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t s = (size_t)y * nx + x;
            /* Density gradient at time t by central differences (Sec. 4). */
            double gx = (L->R[(size_t)y * nx + wrap(x + 1, nx)] -
                         L->R[(size_t)y * nx + wrap(x - 1, nx)]) / 2.0;
            double gy = (L->R[(size_t)wrap(y + 1, ny) * nx + x] -
                         L->R[(size_t)wrap(y - 1, ny) * nx + x]) / 2.0;
            double feq[9], src[9];
            model_equilibrium(L, L->R[s], L->UX[s], L->UY[s], feq);
            /* alpha at this site (a c2 field), else the lattice's;
             * the equilibrium model has no source term */
            double alpha = L->A ? L->A[s] : L->alpha;
            lbmref_source(L->model == LBMREF_MODEL_EQUILIBRIUM ? 0.0 : alpha, gx, gy, src);
            for (int i = 0; i < 9; ++i) {
                /* Right-hand side of Eq. 5 added to f_i(x, t) ... */
                double fi = L->f[i * n + s];
                double fstar = fi - (fi - feq[i]) / L->tau + src[i];
                if (xbc && (x == 0 || x == nx - 1)) {
                    /* a boundary column emits its equilibrium; across the
                     * cut seam the entered column's equilibrium arrives */
                    int crosses = (x == 0 && e[2 * i] < 0) || (x == nx - 1 && e[2 * i] > 0);
                    const double* own = x == 0 ? fin : fout;
                    const double* entered = x == 0 ? fout : fin;
                    fstar = crosses ? entered[i] : own[i];
                }
                /* ... lands at x + e_i at time t + 1 (left-hand side). */
                int xd = wrap(x + e[2 * i], nx);
                int yd = wrap(y + e[2 * i + 1], ny);
                L->fnew[i * n + (size_t)yd * nx + xd] = fstar;
            }
        }
    }
    double* tmp = L->f;
    L->f = L->fnew;
    L->fnew = tmp;
    L->t += 1;
}

int lbmref_step(lbmref* L, int n)
{
    if (!L || n < 0) return LBMREF_EINVAL;
    if (!L->ready) return LBMREF_ESTATE;
    for (int k = 0; k < n; ++k) step_once(L);
    return LBMREF_OK;
}

/* Neumaier's compensated summation, one term at a time. */
static void neumaier_add(double* sum, double* comp, double v)
{
    double t = *sum + v;
    if (fabs(*sum) >= fabs(v))
        *comp += (*sum - t) + v;
    else
        *comp += (v - t) + *sum;
    *sum = t;
}

int lbmref_moments(lbmref* L, double* rho, double* ux, double* uy, double totals[3])
{
    if (!L) return LBMREF_EINVAL;
    if (!L->ready) return LBMREF_ESTATE;
    const int* e = E;
    compute_moments(L);
    size_t n = (size_t)L->nx * L->ny;
    if (rho) memcpy(rho, L->R, n * sizeof(double));
    if (ux) memcpy(ux, L->UX, n * sizeof(double));
    if (uy) memcpy(uy, L->UY, n * sizeof(double));
    double sum[3] = {0, 0, 0}, comp[3] = {0, 0, 0};
    for (size_t s = 0; s < n; ++s) {
        double r = 0.0, jx = 0.0, jy = 0.0;
        for (int i = 0; i < 9; ++i) {
            double fi = L->f[i * n + s];
            r += fi;
            jx += fi * e[2 * i];
            jy += fi * e[2 * i + 1];
        }
        neumaier_add(&sum[0], &comp[0], r);
        neumaier_add(&sum[1], &comp[1], jx);
        neumaier_add(&sum[2], &comp[2], jy);
    }
    int finite = 1;
    for (int k = 0; k < 3; ++k) {
        double v = sum[k] + comp[k];
        if (totals) totals[k] = v;
        if (!isfinite(v)) finite = 0;
    }
    return finite ? LBMREF_OK : LBMREF_ENONFINITE;
}

int lbmref_get_f(lbmref* L, double* f)
{
    if (!L || !f) return LBMREF_EINVAL;
    if (!L->ready) return LBMREF_ESTATE;
    memcpy(f, L->f, 9 * (size_t)L->nx * L->ny * sizeof(double));
    return LBMREF_OK;
}

int lbmref_set_f(lbmref* L, const double* f)
{
    if (!L || !f) return LBMREF_EINVAL;
    memcpy(L->f, f, 9 * (size_t)L->nx * L->ny * sizeof(double));
    L->t = 0;
    L->ready = 1;
    return LBMREF_OK;
}

long long lbmref_time(const lbmref* L) { return L ? L->t : -1; }

void lbmref_set_threads(int n)
{
#ifdef _OPENMP
    if (n <= 0) n = omp_get_num_procs();
    omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int lbmref_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

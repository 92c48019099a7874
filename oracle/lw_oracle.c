/*
 * lw_oracle.c -- plain, serial oracle of the Lienard-Wiechert hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only tests/, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header, constant or helper with the HIP
 * path.  It is written for a reader checking it against the paper by eye:
 * every quantity is computed the direct way, with no blocking, fusion or
 * reordering.
 *
 * Working precision.  The source is compiled twice: with OR_REAL = double
 * (the FP64 oracle) and with OR_REAL = long double (x87 extended precision,
 * a 64-bit significand).  Inputs and outputs are double in both builds; only
 * the arithmetic in between differs.  The extended build arbitrates where the
 * FP64 oracle itself loses digits: the drive of a distant dipole is the
 * difference of its two charges' nearly equal fields, so its rounding relative
 * to the net field grows with the ratio of separation to charge offset.
 *
 * What it computes (arXiv 2107.12437, "PyCharge"):
 *   - parametric point-charge trajectories x(t), y(t), z(t) with exact
 *     derivatives (Sec. 3.1, "Electromagnetic sources");
 *   - the retarded time of Eq. (ret_t), t' = t - R(t')/c, by plain bisection
 *     on tau = t - t' (Sec. 2.2 says only that a root finder is used; the root
 *     is unique for subluminal motion, so the solver does not change the
 *     answer);
 *   - the potentials of Eqs. (V) and (A), the total / Coulomb / radiation
 *     electric field of Eqs. (E), (ECoulomb), (Eradiation) and the magnetic
 *     field of Eq. (B);
 *   - superposition over charges (Sec. 2.2) with a Neumaier-compensated sum;
 *   - the self-consistent Lorentz-oscillator run of Algorithm 1 (Sec. 3.2):
 *     Eq. (LO_equation) with gamma_0 of Sec. 2.3, RK4 steps, dipole charges
 *     placed by Eqs. (r_1), (r_2), stored kinematics linearly interpolated
 *     between steps, dipoles static for t <= 0, own dipole excluded from
 *     the drive, the c/100 speed limit, and the energy of Eq. (dipoleE).
 *
 * Readings where the paper is silent or garbled are stated at the point of use.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <tgmath.h>

#ifndef OR_REAL
#define OR_REAL double
#endif
typedef OR_REAL real;

/* decimal constants read at the working precision */
#ifdef OR_LONG
#define RL(x) x##L
#else
#define RL(x) x
#endif

/* CODATA 2018 (the scipy.constants values of the paper's time). */
#define OR_C     RL(299792458.0)
#define OR_EPS0  RL(8.8541878128e-12)
#define OR_PI    RL(3.14159265358979323846264338327950288)

enum { OR_STATIONARY = 0, OR_UNIFORM_VELOCITY = 1, OR_LINEAR_OSC = 2, OR_CIRCULAR = 3, OR_ACCEL = 4 };
enum { OR_TOTAL = 0, OR_COULOMB = 1, OR_RADIATION = 2 };
enum { OR_OK = 0, OR_E_INVALID = 1, OR_E_SUPERLUMINAL = 2, OR_E_DT_TOO_LARGE = 3,
       OR_E_VELOCITY = 4, OR_E_NOCONV = 5, OR_E_NOMEM = 7, OR_E_NONFINITE = 8 };
enum { OR_FLAG_MASKED = 1u, OR_FLAG_NOCONV = 2u };

/* One point charge with a parametric trajectory (the paper's Charge subclasses). */
typedef struct {
    int32_t kind;
    int32_t pad_;
    double q;
    double c0[3];
    double e1[3];
    double e2[3];
    double amp;
    double omega;
    double phase;
    double accel;
    double v[3];
} or_traj;

/* Size of the working precision's significand in bits (53 or 64). */
int or_real_digits(void)
{
    real x = 1, e = 1;
    int n = 0;
    while (x + e != x) { e /= 2; ++n; }
    return n;
}

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                      */
/* ------------------------------------------------------------------------ */

static real dot3(const real a[3], const real b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3(const real a[3], const real b[3], real out[3])
{
    real r0 = a[1] * b[2] - a[2] * b[1];
    real r1 = a[2] * b[0] - a[0] * b[2];
    real r2 = a[0] * b[1] - a[1] * b[0];
    out[0] = r0; out[1] = r1; out[2] = r2;
}

static real norm3(const real a[3]) { return sqrt(dot3(a, a)); }

static real norm3d(const double a[3])
{
    real b[3];
    b[0] = a[0]; b[1] = a[1]; b[2] = a[2];
    return norm3(b);
}

/* ------------------------------------------------------------------------ */
/* trajectories (Sec. 3.1)                                                   */
/* ------------------------------------------------------------------------ */

/* Position, velocity, acceleration and jerk of a charge at time t.  The paper
 * differentiates trajectories by finite differences unless the user gives
 * exact derivatives; the oracle uses the exact ones. */
static int traj_kin(const or_traj *s, real t, real r[3], real v[3], real a[3], real j[3])
{
    int k;
    for (k = 0; k < 3; ++k) { r[k] = s->c0[k]; v[k] = 0; a[k] = 0; j[k] = 0; }
    switch (s->kind) {
    case OR_STATIONARY:
        return OR_OK;
    case OR_UNIFORM_VELOCITY:
        for (k = 0; k < 3; ++k) { r[k] = s->c0[k] + s->v[k] * t; v[k] = s->v[k]; }
        return OR_OK;
    case OR_LINEAR_OSC: {
        /* r = c0 + A cos(w t + phi) e1 */
        real w = s->omega, A = s->amp;
        real th = w * t + s->phase;
        real c = cos(th), sn = sin(th);
        for (k = 0; k < 3; ++k) {
            r[k] = s->c0[k] + A * c * s->e1[k];
            v[k] = -A * w * sn * s->e1[k];
            a[k] = -A * w * w * c * s->e1[k];
            j[k] = A * w * w * w * sn * s->e1[k];
        }
        return OR_OK;
    }
    case OR_CIRCULAR: {
        /* r = c0 + A (cos(w t + phi) e1 + sin(w t + phi) e2) */
        real w = s->omega, A = s->amp;
        real th = w * t + s->phase;
        real c = cos(th), sn = sin(th);
        for (k = 0; k < 3; ++k) {
            r[k] = s->c0[k] + A * (c * s->e1[k] + sn * s->e2[k]);
            v[k] = A * w * (-sn * s->e1[k] + c * s->e2[k]);
            a[k] = -A * w * w * (c * s->e1[k] + sn * s->e2[k]);
            j[k] = -A * w * w * w * (-sn * s->e1[k] + c * s->e2[k]);
        }
        return OR_OK;
    }
    case OR_ACCEL:
        /* at rest at c0 for t < 0, then r = c0 + (1/2) a t^2 e1 */
        if (t >= 0) {
            for (k = 0; k < 3; ++k) {
                r[k] = s->c0[k] + RL(0.5) * s->accel * t * t * s->e1[k];
                v[k] = s->accel * t * s->e1[k];
                a[k] = s->accel * s->e1[k];
            }
        }
        return OR_OK;
    default:
        return OR_E_INVALID;
    }
}

int or_traj_kin(const or_traj *s, double t, double r[3], double v[3], double a[3], double j[3])
{
    real rr[3], vv[3], aa[3], jj[3];
    int k, st = traj_kin(s, t, rr, vv, aa, jj);
    for (k = 0; k < 3; ++k) { r[k] = rr[k]; v[k] = vv[k]; a[k] = aa[k]; j[k] = jj[k]; }
    return st;
}

/* Largest speed the charge can have at any time <= t. */
static real traj_vmax(const or_traj *s, real t)
{
    switch (s->kind) {
    case OR_UNIFORM_VELOCITY: return norm3d(s->v);
    case OR_LINEAR_OSC:
    case OR_CIRCULAR: return fabs((real)s->amp * s->omega);
    case OR_ACCEL: return t > 0 ? fabs((real)s->accel) * t : 0;
    default: return 0;
    }
}

/* ------------------------------------------------------------------------ */
/* retarded time, Eq. (ret_t)                                                */
/* ------------------------------------------------------------------------ */

/* g(tau) = c tau - |x - r(t - tau)|; its root is t - t'. */
static real ret_g(const or_traj *s, const real x[3], real t, real tau)
{
    real r[3], v[3], a[3], j[3], d[3];
    traj_kin(s, t - tau, r, v, a, j);
    d[0] = x[0] - r[0]; d[1] = x[1] - r[1]; d[2] = x[2] - r[2];
    return OR_C * tau - norm3(d);
}

/* Bisection down to two adjacent numbers of the working precision.  For
 * |v| <= vmax < c the distance |x - r(t - tau)| moves by at most vmax * tau
 * from its value D0 at tau = 0, so the root lies in [D0/(c + vmax),
 * D0/(c - vmax)].  Returns the end of the final bracket with the smaller |g|. */
static int retarded_tau(const or_traj *s, const real x[3], real t, real *tau_out, int *iters_out)
{
    real r[3], v[3], a[3], j[3], d[3], D0, vmax, lo, hi, glo, ghi;
    int it = 0, grow = 0;
    traj_kin(s, t, r, v, a, j);
    d[0] = x[0] - r[0]; d[1] = x[1] - r[1]; d[2] = x[2] - r[2];
    D0 = norm3(d);
    vmax = traj_vmax(s, t);
    if (!(vmax < OR_C)) return OR_E_SUPERLUMINAL;
    if (D0 == 0) { *tau_out = 0; if (iters_out) *iters_out = 0; return OR_OK; }
    lo = D0 / (OR_C + vmax);
    hi = D0 / (OR_C - vmax);
    /* guard the bracket against rounding at its ends */
    if (ret_g(s, x, t, lo) > 0) lo = 0;
    while (ret_g(s, x, t, hi) < 0) {
        hi *= 2;
        if (++grow > 64) return OR_E_NOCONV;
    }
    for (;;) {
        real mid = lo + RL(0.5) * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        if (ret_g(s, x, t, mid) < 0) lo = mid; else hi = mid;
        if (++it > 4000) return OR_E_NOCONV;
    }
    glo = fabs(ret_g(s, x, t, lo));
    ghi = fabs(ret_g(s, x, t, hi));
    *tau_out = (glo <= ghi) ? lo : hi;
    if (iters_out) *iters_out = it;
    return OR_OK;
}

int or_retarded_tau(const or_traj *s, const double x[3], double t, double *tau_out, int *iters_out)
{
    real xx[3], tau = 0;
    int st;
    xx[0] = x[0]; xx[1] = x[1]; xx[2] = x[2];
    st = retarded_tau(s, xx, t, &tau, iters_out);
    if (st == OR_OK) *tau_out = tau;
    return st;
}

/* ------------------------------------------------------------------------ */
/* Lienard-Wiechert potentials and fields of one charge                      */
/* ------------------------------------------------------------------------ */

/* Evaluates, at the retarded time of charge s seen from x at time t,
 *   out[0]   = Phi               Eq. (V)
 *   out[1:4] = A                 Eq. (A), SI form mu0 q c beta / (4 pi kappa R)
 *   out[4:7] = E                 Eq. (E) (or Eq. (ECoulomb) / Eq. (Eradiation))
 *   out[7:10]= B = n x E / c     Eq. (B), using the same E kind.
 * Eq. (A) is printed with beta where SI units need c*beta = v (the Gaussian
 * form of Jackson carried into SI); the oracle uses the SI form, which makes
 * A = Phi * beta / c.  Returns OR_FLAG_MASKED when the retarded distance is
 * below mask_r (out is then left untouched). */
static unsigned lw_pair(const or_traj *s, const real x[3], real t, int field_kind, real mask_r, real out[10])
{
    real tau, tp, r[3], v[3], a[3], j[3];
    real Rv[3], R, n[3], beta[3], bdot[3], kappa, K, nmb[3], cr1[3], cr2[3];
    real coul[3], rad[3], E[3], B[3], beta2, phi;
    int k, st;
    st = retarded_tau(s, x, t, &tau, NULL);
    if (st != OR_OK) return OR_FLAG_NOCONV;
    tp = t - tau;
    traj_kin(s, tp, r, v, a, j);
    for (k = 0; k < 3; ++k) Rv[k] = x[k] - r[k];
    R = norm3(Rv);
    if (!(R >= mask_r) || R == 0) return OR_FLAG_MASKED;
    for (k = 0; k < 3; ++k) {
        n[k] = Rv[k] / R;
        beta[k] = v[k] / OR_C;
        bdot[k] = a[k] / OR_C;      /* d(beta)/dt' */
        nmb[k] = n[k] - beta[k];
    }
    kappa = 1 - dot3(n, beta);
    beta2 = dot3(beta, beta);
    K = s->q / (4 * OR_PI * OR_EPS0);
    phi = K / (kappa * R);
    /* Coulomb (velocity) field */
    for (k = 0; k < 3; ++k)
        coul[k] = K * nmb[k] * (1 - beta2) / (kappa * kappa * kappa * R * R);
    /* radiation (acceleration) field: n x ((n - beta) x beta_dot) / (c kappa^3 R) */
    cross3(nmb, bdot, cr1);
    cross3(n, cr1, cr2);
    for (k = 0; k < 3; ++k)
        rad[k] = K * cr2[k] / (OR_C * kappa * kappa * kappa * R);
    for (k = 0; k < 3; ++k) {
        if (field_kind == OR_COULOMB) E[k] = coul[k];
        else if (field_kind == OR_RADIATION) E[k] = rad[k];
        else E[k] = coul[k] + rad[k];
    }
    cross3(n, E, B);
    out[0] = phi;
    for (k = 0; k < 3; ++k) {
        out[1 + k] = phi * beta[k] / OR_C;
        out[4 + k] = E[k];
        out[7 + k] = B[k] / OR_C;
    }
    return 0u;
}

unsigned or_lw_pair(const or_traj *s, const double x[3], double t, int field_kind, double mask_r, double out[10])
{
    real xx[3], o[10];
    unsigned f;
    int k;
    xx[0] = x[0]; xx[1] = x[1]; xx[2] = x[2];
    f = lw_pair(s, xx, t, field_kind, mask_r, o);
    if (!f)
        for (k = 0; k < 10; ++k) out[k] = o[k];
    return f;
}

/* Neumaier (improved Kahan) summation step. */
static void neumaier_add(real *sum, real *comp, real x)
{
    real t = *sum + x;
    if (fabs(*sum) >= fabs(x)) *comp += (*sum - t) + x;
    else *comp += (x - t) + *sum;
    *sum = t;
}

/* Superposition over all charges for every (time, point).
 * pts is SoA [3][n_pts]; out is [n_times][10][n_pts]; flags (nullable) is
 * per point, OR-ed over times.  A (point, time) whose retarded distance to any
 * charge is below mask_r gets NaN in all ten outputs. */
int or_fields(const or_traj *ch, int n_ch, const double *pts, int64_t n_pts, const double *times,
              int n_times, int field_kind, double mask_r, double *out, uint32_t *flags)
{
    int64_t p;
    int ti, c, k;
    if (n_ch < 0 || n_pts < 0 || n_times < 0) return OR_E_INVALID;
    for (c = 0; c < n_ch; ++c)
        for (ti = 0; ti < n_times; ++ti)
            if (!(traj_vmax(&ch[c], times[ti]) < OR_C)) return OR_E_SUPERLUMINAL;
    if (flags) memset(flags, 0, sizeof(uint32_t) * (size_t)n_pts);
    for (ti = 0; ti < n_times; ++ti) {
        for (p = 0; p < n_pts; ++p) {
            real x[3], sum[10], comp[10], one[10];
            unsigned fl = 0u;
            x[0] = pts[p]; x[1] = pts[n_pts + p]; x[2] = pts[2 * n_pts + p];
            for (k = 0; k < 10; ++k) { sum[k] = 0; comp[k] = 0; }
            for (c = 0; c < n_ch; ++c) {
                unsigned f = lw_pair(&ch[c], x, times[ti], field_kind, mask_r, one);
                fl |= f;
                if (f) continue;
                for (k = 0; k < 10; ++k) neumaier_add(&sum[k], &comp[k], one[k]);
            }
            for (k = 0; k < 10; ++k) {
                double val = (fl & OR_FLAG_MASKED) ? (double)NAN : (double)(sum[k] + comp[k]);
                out[((int64_t)ti * 10 + k) * n_pts + p] = val;
            }
            if (flags) flags[p] |= fl;
        }
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Lorentz oscillators (Sec. 2.3, Algorithm 1)                               */
/* ------------------------------------------------------------------------ */

enum { OR_DT_STRICT = 0, OR_DT_EXTRAPOLATE = 1 };

typedef struct {
    int n_dip;
    const double *origin, *axis, *q;
    const double *mamp, *momega, *mphase;  /* origin motion O + mamp cos(momega t + mphase), or NULL */
    const double *d0;
    real *coef_p, *coef_m;     /* m2/(m1+m2), -m1/(m1+m2): charge offsets per unit r_dip */
    real *hist;                /* [(steps+1)][n_dip][3] = (d, d_dot, d_ddot) */
    real dt;
} or_lo;

/* Stored kinematics (d, d_dot, d_ddot) of dipole jd at time tp, given samples
 * 0..n.  Before t = 0 the dipole is static at d0 (Sec. 3.2: dipoles only start
 * to oscillate after the first step).  Between samples each of the three is
 * interpolated linearly (Sec. 3.1).  Beyond the newest sample n (only reached
 * when dt exceeds the light travel time between dipoles) the reading is a
 * second-order Taylor step from sample n. */
static void lo_hist_at(const or_lo *L, int jd, int64_t n, real tp, real out[3])
{
    const real *h;
    real s, u, tau;
    int64_t k;
    if (tp < 0) { out[0] = L->d0[jd]; out[1] = 0; out[2] = 0; return; }
    s = tp / L->dt;
    k = (int64_t)floor(s);
    if (k >= n) {
        h = &L->hist[(n * L->n_dip + jd) * 3];
        tau = tp - (real)n * L->dt;
        out[0] = h[0] + h[1] * tau + RL(0.5) * h[2] * tau * tau;
        out[1] = h[1] + h[2] * tau;
        out[2] = h[2];
        return;
    }
    u = s - (real)k;
    {
        const real *h0 = &L->hist[(k * L->n_dip + jd) * 3];
        const real *h1 = &L->hist[((k + 1) * L->n_dip + jd) * 3];
        out[0] = (1 - u) * h0[0] + u * h1[0];
        out[1] = (1 - u) * h0[1] + u * h1[1];
        out[2] = (1 - u) * h0[2] + u * h1[2];
    }
}

/* A caller's double history [(n+1)][n_dip][3] in the working precision. */
static real *hist_copy(const double *hist, int64_t n, int n_dip)
{
    size_t m = 3 * (size_t)(n + 1) * (size_t)n_dip, i;
    real *h = (real *)malloc(sizeof(real) * (m ? m : 1));
    if (h)
        for (i = 0; i < m; ++i) h[i] = hist[i];
    return h;
}

/* The history reading above on its own, for tests: hist holds samples 0..n of
 * n_dip dipoles as [(n+1)][n_dip][3]; d0 the moments before t = 0. */
int or_hist_at(const double *hist, int n_dip, int jd, int64_t n, double dt, const double *d0, double tp,
               double out[3])
{
    or_lo L;
    real o[3];
    if (n_dip <= 0 || jd < 0 || jd >= n_dip || n < 0 || !(dt > 0.0)) return OR_E_INVALID;
    memset(&L, 0, sizeof(L));
    L.n_dip = n_dip; L.dt = dt; L.d0 = d0;
    L.hist = hist_copy(hist, n, n_dip);
    if (!L.hist) return OR_E_NOMEM;
    lo_hist_at(&L, jd, n, tp, o);
    out[0] = o[0]; out[1] = o[1]; out[2] = o[2];
    free(L.hist);
    return OR_OK;
}

/* Origin (centre of mass) of dipole jd at time t and its velocity and
 * acceleration: fixed, or moving as O + m cos(w t + phi) (Sec. 4.3, moving
 * dipoles; the motion is prescribed for all t, before t = 0 as well). */
static void lo_origin(const or_lo *L, int jd, real t, real R[3], real V[3], real A[3])
{
    int k;
    real c = 1, s = 0, w = 0;
    if (L->mamp) {
        w = L->momega[jd];
        c = cos(w * t + L->mphase[jd]);
        s = sin(w * t + L->mphase[jd]);
    }
    for (k = 0; k < 3; ++k) {
        real m = L->mamp ? L->mamp[jd * 3 + k] : 0;
        R[k] = L->origin[jd * 3 + k] + m * c;
        V[k] = -w * m * s;
        A[k] = -w * w * m * c;
    }
}

/* Position, velocity, acceleration of charge `which` (0: +q at the positive end,
 * 1: -q) of dipole jd at time tp, by Eqs. (r_1), (r_2) with r_dip = (d/q) p
 * about the dipole's origin at tp. */
static void lo_charge_kin(const or_lo *L, int jd, int which, int64_t n, real tp,
                          real r[3], real v[3], real a[3])
{
    real h[3], cf, R[3], V[3], A[3];
    int k;
    lo_hist_at(L, jd, n, tp, h);
    lo_origin(L, jd, tp, R, V, A);
    cf = (which == 0 ? L->coef_p[jd] : L->coef_m[jd]) / L->q[jd];
    for (k = 0; k < 3; ++k) {
        real p = L->axis[jd * 3 + k];
        r[k] = R[k] + cf * h[0] * p;
        v[k] = V[k] + cf * h[1] * p;
        a[k] = A[k] + cf * h[2] * p;
    }
}

static real lo_g(const or_lo *L, int jd, int which, int64_t n, const real x[3], real t, real tau)
{
    real r[3], v[3], a[3], d[3];
    lo_charge_kin(L, jd, which, n, t - tau, r, v, a);
    d[0] = x[0] - r[0]; d[1] = x[1] - r[1]; d[2] = x[2] - r[2];
    return OR_C * tau - norm3(d);
}

/* Total LW electric field (Eq. (E)) at x, time t, of charge `which` of dipole jd. */
static int lo_charge_field(const or_lo *L, int jd, int which, int64_t n, const real x[3], real t,
                           real E[3])
{
    real lo = 0, hi, tau, r[3], v[3], a[3], Rv[3], R, nn[3], beta[3], bdot[3], nmb[3];
    real cr1[3], cr2[3], kappa, beta2, K, qc;
    int k, grow = 0, it = 0;
    {
        real O[3], V[3], A[3];
        lo_origin(L, jd, t, O, V, A);
        for (k = 0; k < 3; ++k) Rv[k] = x[k] - O[k];
    }
    hi = 2 * norm3(Rv) / OR_C;
    if (hi <= 0) return OR_E_INVALID;
    while (lo_g(L, jd, which, n, x, t, hi) < 0) { hi *= 2; if (++grow > 64) return OR_E_NOCONV; }
    for (;;) {
        real mid = lo + RL(0.5) * (hi - lo);
        if (!(mid > lo && mid < hi)) break;
        if (lo_g(L, jd, which, n, x, t, mid) < 0) lo = mid; else hi = mid;
        if (++it > 4000) return OR_E_NOCONV;
    }
    tau = fabs(lo_g(L, jd, which, n, x, t, lo)) <= fabs(lo_g(L, jd, which, n, x, t, hi)) ? lo : hi;
    lo_charge_kin(L, jd, which, n, t - tau, r, v, a);
    for (k = 0; k < 3; ++k) Rv[k] = x[k] - r[k];
    R = norm3(Rv);
    for (k = 0; k < 3; ++k) {
        nn[k] = Rv[k] / R;
        beta[k] = v[k] / OR_C;
        bdot[k] = a[k] / OR_C;
        nmb[k] = nn[k] - beta[k];
    }
    kappa = 1 - dot3(nn, beta);
    beta2 = dot3(beta, beta);
    qc = (which == 0) ? L->q[jd] : -L->q[jd];
    K = qc / (4 * OR_PI * OR_EPS0);
    cross3(nmb, bdot, cr1);
    cross3(nn, cr1, cr2);
    for (k = 0; k < 3; ++k)
        E[k] = K * nmb[k] * (1 - beta2) / (kappa * kappa * kappa * R * R)
             + K * cr2[k] / (OR_C * kappa * kappa * kappa * R);
    return OR_OK;
}

/* Drive field E_d of dipole i at time t: the component along its axis of the
 * total field at its origin of every charge of the other dipoles of the same
 * instance [i_lo, i_hi) (Eq. (LO_equation); own dipole excluded, Sec. 3.2). */
static int lo_drive(const or_lo *L, int i, int i_lo, int i_hi, int64_t n, real t, real *Ed)
{
    real sum = 0, comp = 0, E[3], x[3], V[3], A[3], p[3];
    int jd, w, st;
    lo_origin(L, i, t, x, V, A);                 /* the field is taken at the origin at time t */
    p[0] = L->axis[i * 3]; p[1] = L->axis[i * 3 + 1]; p[2] = L->axis[i * 3 + 2];
    for (jd = i_lo; jd < i_hi; ++jd) {
        if (jd == i) continue;
        for (w = 0; w < 2; ++w) {
            st = lo_charge_field(L, jd, w, n, x, t, E);
            if (st != OR_OK) return st;
            neumaier_add(&sum, &comp, dot3(E, p));
        }
    }
    *Ed = sum + comp;
    return OR_OK;
}

/* Self-consistent run of independent instances (CSR offsets inst_off[0..n_inst]).
 * State of dipole i: moment d (scalar along its fixed axis) and d_dot.  Each step
 * is one classic RK4 step of
 *     d'' + gamma0 d' + omega0^2 d = (q^2/m) E_d(t),
 *     gamma0 = q^2 omega0^2 / (6 pi eps0 c^3 m),   m = m1 m2 / (m1 + m2),
 * with E_d at the stage times t_n, t_n + dt/2 (stages 2 and 3) and t_n + dt,
 * all taken from the stored history up to sample n; all dipoles then advance
 * together (the update order of Algorithm 2).  Sample n+1 stores
 * (d, d_dot, d_ddot) with d_ddot from the equation of motion at t_{n+1}; E_d at
 * t_{n+1} is reused as the first stage of the next step.  Sample 0 is
 * (d0, 0, d_ddot(0)).
 * Outputs every out_stride steps (n_out = steps/out_stride + 1 rows of n_dip):
 * moment d, d_dot, energy of Eq. (dipoleE), drive field E_d, and since t = 0
 * the work done on the dipole by its drive field (integral of E_d d_dot) and
 * the energy it radiated (integral of the Larmor power |d_ddot|^2/(6 pi eps0
 * c^3)), both by the trapezoid rule over steps (Sec. 2.5: the sum over dipoles
 * of energy - absorbed + radiated is the conserved W_total).  Any may be NULL. */
int or_dipole_run(int n_dip, const double *origin, const double *axis, const double *omega0,
                  const double *q, const double *m1, const double *m2, const double *d0,
                  const double *mamp, const double *momega, const double *mphase,
                  int n_inst, const int32_t *inst_off, double dt, int64_t steps, int policy,
                  double max_vel, int64_t out_stride,
                  double *out_d, double *out_v, double *out_E, double *out_Ed, double *out_Wabs,
                  double *out_Wrad, double *hist_out)
{
    or_lo L;
    real *mass, *gam, *Ecur, *Emid, *Eend, *ynew, *Wabs, *Wrad;
    /* Larmor power of a dipole, |d_ddot|^2 / (6 pi eps0 c^3) (Sec. 2.5) */
    const real KLAR = 1 / (6 * OR_PI * OR_EPS0 * OR_C * OR_C * OR_C);
    const real h_dt = dt;
    int i, inst, st = OR_OK;
    int64_t n, nstore;
    if (n_dip <= 0 || n_inst <= 0 || inst_off[0] != 0 || inst_off[n_inst] != n_dip || !(dt > 0.0) ||
        steps < 0 || out_stride <= 0)
        return OR_E_INVALID;
    for (inst = 0; inst < n_inst; ++inst)
        if (inst_off[inst + 1] < inst_off[inst]) return OR_E_INVALID;
    if (mamp)
        for (i = 0; i < n_dip; ++i)       /* a moving origin needs a frequency; a fixed offset belongs in origin */
            if (norm3d(&mamp[i * 3]) > 0 && momega[i] == 0.0) return OR_E_INVALID;
    if (policy == OR_DT_STRICT) {
        /* Sec. 3.2: radiation must not reach another dipole within one step */
        for (inst = 0; inst < n_inst; ++inst) {
            int a, b;
            for (a = inst_off[inst]; a < inst_off[inst + 1]; ++a)
                for (b = a + 1; b < inst_off[inst + 1]; ++b) {
                    real d[3];
                    real low;
                    d[0] = (real)origin[a * 3] - origin[b * 3];
                    d[1] = (real)origin[a * 3 + 1] - origin[b * 3 + 1];
                    d[2] = (real)origin[a * 3 + 2] - origin[b * 3 + 2];
                    /* moving origins: the separation never falls below this */
                    low = norm3(d) - (mamp ? norm3d(&mamp[a * 3]) + norm3d(&mamp[b * 3]) : 0);
                    if (!(OR_C * h_dt < low)) return OR_E_DT_TOO_LARGE;
                }
        }
    }
    nstore = steps + 1;
    L.n_dip = n_dip; L.origin = origin; L.axis = axis; L.q = q; L.d0 = d0; L.dt = dt;
    L.mamp = mamp; L.momega = momega; L.mphase = mphase;
    L.hist = (real *)malloc(sizeof(real) * 3 * (size_t)nstore * (size_t)n_dip);
    L.coef_p = (real *)malloc(sizeof(real) * (size_t)n_dip);
    L.coef_m = (real *)malloc(sizeof(real) * (size_t)n_dip);
    mass = (real *)malloc(sizeof(real) * (size_t)n_dip);
    gam = (real *)malloc(sizeof(real) * (size_t)n_dip);
    Ecur = (real *)malloc(sizeof(real) * (size_t)n_dip);
    Emid = (real *)malloc(sizeof(real) * (size_t)n_dip);
    Eend = (real *)malloc(sizeof(real) * (size_t)n_dip);
    ynew = (real *)malloc(sizeof(real) * 2 * (size_t)n_dip);
    Wabs = (real *)calloc((size_t)n_dip, sizeof(real));
    Wrad = (real *)calloc((size_t)n_dip, sizeof(real));
    if (!L.hist || !L.coef_p || !L.coef_m || !mass || !gam || !Ecur || !Emid || !Eend || !ynew || !Wabs || !Wrad) {
        st = OR_E_NOMEM;
        goto done;
    }
    for (i = 0; i < n_dip; ++i) {
        real M = (real)m1[i] + m2[i];
        mass[i] = (real)m1[i] * m2[i] / M;                              /* Eq. (eff_mass) */
        gam[i] = (real)q[i] * q[i] * omega0[i] * omega0[i] /
                 (6 * OR_PI * OR_EPS0 * OR_C * OR_C * OR_C * mass[i]);   /* gamma_0, Sec. 2.3 */
        L.coef_p[i] = m2[i] / M;                                         /* Eq. (r_1) */
        L.coef_m[i] = -m1[i] / M;                                        /* Eq. (r_2) */
    }
    /* t = 0: drive from the static pre-history, then sample 0 */
    for (inst = 0; inst < n_inst; ++inst)
        for (i = inst_off[inst]; i < inst_off[inst + 1]; ++i) {
            st = lo_drive(&L, i, inst_off[inst], inst_off[inst + 1], 0, 0, &Ecur[i]);
            if (st) goto done;
        }
    for (i = 0; i < n_dip; ++i) {
        real *h = &L.hist[(size_t)i * 3];
        h[0] = d0[i];
        h[1] = 0;
        h[2] = (real)q[i] * q[i] / mass[i] * Ecur[i] - (real)omega0[i] * omega0[i] * d0[i];
    }
    for (n = 0;; ++n) {
        if (n % out_stride == 0) {
            int64_t row = n / out_stride;
            for (i = 0; i < n_dip; ++i) {
                const real *h = &L.hist[(n * n_dip + i) * 3];
                if (out_d) out_d[row * n_dip + i] = h[0];
                if (out_v) out_v[row * n_dip + i] = h[1];
                if (out_E) out_E[row * n_dip + i] =
                    mass[i] / (2 * (real)q[i] * q[i]) * ((real)omega0[i] * omega0[i] * h[0] * h[0] + h[1] * h[1]);
                if (out_Ed) out_Ed[row * n_dip + i] = Ecur[i];
                if (out_Wabs) out_Wabs[row * n_dip + i] = Wabs[i];
                if (out_Wrad) out_Wrad[row * n_dip + i] = Wrad[i];
            }
        }
        if (n == steps) break;
        {
            real t = (real)n * h_dt;
            for (inst = 0; inst < n_inst; ++inst)
                for (i = inst_off[inst]; i < inst_off[inst + 1]; ++i) {
                    st = lo_drive(&L, i, inst_off[inst], inst_off[inst + 1], n, t + RL(0.5) * h_dt, &Emid[i]);
                    if (st) goto done;
                    st = lo_drive(&L, i, inst_off[inst], inst_off[inst + 1], n, t + h_dt, &Eend[i]);
                    if (st) goto done;
                }
        }
        for (i = 0; i < n_dip; ++i) {
            const real *h = &L.hist[(n * n_dip + i) * 3];
            real w2 = (real)omega0[i] * omega0[i], g = gam[i], f = (real)q[i] * q[i] / mass[i];
            real y0 = h[0], y1 = h[1];
            /* f(y, E) = (y1, f E - g y1 - w2 y0) */
            real k1d = y1, k1v = f * Ecur[i] - g * y1 - w2 * y0;
            real y0b = y0 + RL(0.5) * h_dt * k1d, y1b = y1 + RL(0.5) * h_dt * k1v;
            real k2d = y1b, k2v = f * Emid[i] - g * y1b - w2 * y0b;
            real y0c = y0 + RL(0.5) * h_dt * k2d, y1c = y1 + RL(0.5) * h_dt * k2v;
            real k3d = y1c, k3v = f * Emid[i] - g * y1c - w2 * y0c;
            real y0d = y0 + h_dt * k3d, y1d = y1 + h_dt * k3v;
            real k4d = y1d, k4v = f * Eend[i] - g * y1d - w2 * y0d;
            ynew[2 * i] = y0 + h_dt / 6 * (k1d + 2 * k2d + 2 * k3d + k4d);
            ynew[2 * i + 1] = y1 + h_dt / 6 * (k1v + 2 * k2v + 2 * k3v + k4v);
        }
        for (i = 0; i < n_dip; ++i) {
            real *h = &L.hist[((n + 1) * n_dip + i) * 3];
            const real *ho = &L.hist[(n * n_dip + i) * 3];
            real speed;
            h[0] = ynew[2 * i];
            h[1] = ynew[2 * i + 1];
            h[2] = (real)q[i] * q[i] / mass[i] * Eend[i] - gam[i] * h[1] - (real)omega0[i] * omega0[i] * h[0];
            /* energy bookkeeping of Sec. 2.5, trapezoid rule over the step: work done
               by the drive field (E_d d_dot) and the Larmor power of the dipole */
            Wabs[i] += RL(0.5) * h_dt * (ho[1] * Ecur[i] + h[1] * Eend[i]);
            Wrad[i] += RL(0.5) * h_dt * KLAR * (ho[2] * ho[2] + h[2] * h[2]);
            Ecur[i] = Eend[i];
            /* the charge speeds are at most |origin velocity| + |coef| * |d_dot| / q;
               Sec. 3.2 raises above max_vel */
            speed = fmax(fabs(L.coef_p[i]), fabs(L.coef_m[i])) * fabs(h[1]) / q[i];
            if (mamp) speed += fabs((real)momega[i]) * norm3d(&mamp[i * 3]);
            if (!(isfinite(h[0]) && isfinite(h[1]) && isfinite(h[2]))) { st = OR_E_NONFINITE; goto done; }
            if (max_vel > 0.0 && speed > max_vel) { st = OR_E_VELOCITY; goto done; }
        }
    }
    if (hist_out) {
        size_t m = 3 * (size_t)nstore * (size_t)n_dip, k;
        for (k = 0; k < m; ++k) hist_out[k] = L.hist[k];
    }
done:
    free(L.hist); free(L.coef_p); free(L.coef_m); free(mass); free(gam);
    free(Ecur); free(Emid); free(Eend); free(ynew); free(Wabs); free(Wrad);
    return st;
}

/* Field of every dipole charge at points pts (SoA [3][n_pts]) and times (all
 * <= steps*dt), from a finished run's history hist ([(steps+1)][n_dip][3]).
 * out is [n_times][3][n_pts] (E only, total field). */
int or_dipole_fields(int n_dip, const double *origin, const double *axis, const double *q,
                     const double *m1, const double *m2, const double *d0,
                     const double *mamp, const double *momega, const double *mphase, double dt, int64_t steps,
                     const double *hist, const double *pts, int64_t n_pts, const double *times,
                     int n_times, double *out)
{
    or_lo L;
    int i, ti, w, k, st = OR_OK;
    int64_t p;
    L.n_dip = n_dip; L.origin = origin; L.axis = axis; L.q = q; L.d0 = d0; L.dt = dt;
    L.mamp = mamp; L.momega = momega; L.mphase = mphase;
    L.hist = hist_copy(hist, steps, n_dip);
    L.coef_p = (real *)malloc(sizeof(real) * (size_t)n_dip);
    L.coef_m = (real *)malloc(sizeof(real) * (size_t)n_dip);
    if (!L.hist || !L.coef_p || !L.coef_m) { st = OR_E_NOMEM; goto done; }
    for (i = 0; i < n_dip; ++i) {
        L.coef_p[i] = m2[i] / ((real)m1[i] + m2[i]);
        L.coef_m[i] = -m1[i] / ((real)m1[i] + m2[i]);
    }
    for (ti = 0; ti < n_times; ++ti) {
        if (!(times[ti] <= (double)steps * dt)) { st = OR_E_INVALID; goto done; }
        for (p = 0; p < n_pts; ++p) {
            real x[3], sum[3] = {0, 0, 0}, comp[3] = {0, 0, 0}, E[3];
            x[0] = pts[p]; x[1] = pts[n_pts + p]; x[2] = pts[2 * n_pts + p];
            for (i = 0; i < n_dip; ++i)
                for (w = 0; w < 2; ++w) {
                    st = lo_charge_field(&L, i, w, steps, x, times[ti], E);
                    if (st) goto done;
                    for (k = 0; k < 3; ++k) neumaier_add(&sum[k], &comp[k], E[k]);
                }
            for (k = 0; k < 3; ++k) out[((int64_t)ti * 3 + k) * n_pts + p] = sum[k] + comp[k];
        }
    }
done:
    free(L.hist); free(L.coef_p); free(L.coef_m);
    return st;
}

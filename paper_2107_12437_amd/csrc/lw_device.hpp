// lw_device.hpp -- device math of the Lienard-Wiechert path for gfx950.
//
// Retarded time (Eq. (ret_t)) by a safeguarded Newton iteration in FP64, the
// retarded kinematics of each trajectory family, and the Lienard-Wiechert
// potentials and fields (Eqs. (V), (A), (E), (ECoulomb), (Eradiation), (B)) in
// the working precision F (float for the mixed path, double for the FP64 path).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lw {

// CODATA 2018
constexpr double C_LIGHT = 299792458.0;
constexpr double INV_C = 1.0 / 299792458.0;
constexpr double EPS0 = 8.8541878128e-12;
constexpr double PI = 3.14159265358979323846;
constexpr double K_COUL = 1.0 / (4.0 * PI * EPS0);

enum { K_STATIONARY = 0, K_UNIFORM_VELOCITY = 1, K_LINEAR_OSC = 2, K_CIRCULAR = 3, K_ACCEL = 4 };
enum { F_TOTAL = 0, F_COULOMB = 1, F_RADIATION = 2 };
enum { FLAG_MASKED = 1u, FLAG_NOCONV = 2u };
enum { OUT_PHI = 1, OUT_A = 2, OUT_E = 4, OUT_B = 8, OUT_S = 16 };

// Per (time, charge) source record, written by the preparation kernel and read
// wave-uniformly (scalar loads) by the field kernels.
struct alignas(16) SrcRec {
    int32_t kind;
    float kqf;        // kq in FP32 (mixed path)
    double kq;        // q / (4 pi eps0)
    double t;         // observation time
    double c0[3];
    double e1[3];
    double e2[3];
    double e3[3];     // e1 x e2
    double amp, omega;  // uniform velocity: c^2 - |v|^2 and its reciprocal (rcp_steer)
    double cT, sT;    // cos, sin of Theta = omega t + phase
    double accel;
    double Lmax;      // accel: distance travelled along e1 by time t
    double v[3];
    double rt[3];     // uniform velocity: position at time t
    // FP32 coefficients of beta and beta_dot (mixed path) in the orbit frame:
    // circular  beta = -s bw1 + c bw2,  beta_dot = -(c aw1 + s aw2);
    // linear    beta = -s bw1,          beta_dot = -c aw1;
    // bw = amp omega / c * e, aw = amp omega^2 / c * e; uniform velocity: bw1 = beta
    float bw1[3], bw2[3], aw1[3], aw2[3];
};

// Retarded kinematics seen from the observation point: R = x - r(t'),
// velocity and acceleration of the charge at t' (Sec. 2.1).
struct Kin {
    double R[3];
    double v[3];        // FP64 path
    double a[3];
    float bf[3], df[3]; // mixed path: beta = v / c and beta_dot = a / c in FP32
    double tp;          // retarded time t'
    double cph, sph;    // cos, sin of the phase at t' (oscillating families)
    uint32_t flags;
    int iters;          // solver iterations taken (ITER_FALLBACK set when the mixed path
                        // fell back to the safeguarded solver); read only by the
                        // iteration-histogram kernels, dead code elsewhere
};

constexpr int ITER_FALLBACK = 1 << 16;

// The mixed path's beta and beta_dot from FP64 velocity and acceleration.
__device__ __forceinline__ void kin_beta_from_va(Kin &k)
{
    for (int i = 0; i < 3; ++i) {
        k.bf[i] = (float)(k.v[i] * INV_C);
        k.df[i] = (float)(k.a[i] * INV_C);
    }
}

// a * b + k with the constant k read from a scalar register pair.  Polynomial
// coefficients used this way stay out of vector registers: held there, every
// accumulate would first need a copy of its coefficient (the two-address form
// overwrites the addend), and the coefficients would take ~30 VGPRs.
__device__ __forceinline__ double fma_k(double a, double b, double k)
{
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(k));
    return r;
}

// sin and cos of a small angle |x| <= 0.75 from their Taylor series (terms
// through x^17 and x^16; the truncation error is below 1e-18).
__device__ __forceinline__ void sincos_small(double x, double &s, double &c)
{
    const double x2 = x * x;
    double ps = fma_k(x2, -1.0 / 355687428096000.0, 1.0 / 1307674368000.0);   // -1/17!, 1/15!
    ps = fma_k(ps, x2, -1.0 / 6227020800.0);       // -1/13!
    ps = fma_k(ps, x2, 1.0 / 39916800.0);          //  1/11!
    ps = fma_k(ps, x2, -1.0 / 362880.0);           // -1/9!
    ps = fma_k(ps, x2, 1.0 / 5040.0);              //  1/7!
    ps = fma_k(ps, x2, -1.0 / 120.0);
    ps = fma_k(ps, x2, 1.0 / 6.0);
    // ps now holds 1/3! - x^2/5! + ...; sin x = x - x^3 * ps
    s = fma(-x * x2, ps, x);
    double pc = fma_k(x2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);       // 1/16!, -1/14!
    pc = fma_k(pc, x2, 1.0 / 479001600.0);         //  1/12!
    pc = fma_k(pc, x2, -1.0 / 3628800.0);          // -1/10!
    pc = fma_k(pc, x2, 1.0 / 40320.0);             //  1/8!
    pc = fma_k(pc, x2, -1.0 / 720.0);              // -1/6!
    pc = fma_k(pc, x2, 1.0 / 24.0);                //  1/4!
    pc = fma(pc, x2, -0.5);                        // -1/2!
    c = fma(pc, x2, 1.0);
}

// sin and cos for |x| < 2^30: x = k pi/2 + r with pi/2 split into three
// doubles (FMA Cody-Waite reduction, |r| <= pi/4), the Taylor kernel on r, then
// the quadrant's swap and signs.
__device__ __forceinline__ void sincos_reduced(double x, double &s, double &c)
{
    const double P1 = 0x1.921fb54442d18p+0;     // pi/2 = P1 + P2 + P3
    const double P2 = 0x1.1a62633145c07p-54;
    const double P3 = -0x1.f1976b7ed8fbcp-110;
    const double k = rint(x * 0x1.45f306dc9c883p-1);   // x * 2/pi
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    r = fma(-k, P3, r);
    double sr, cr;
    sincos_small(r, sr, cr);
    const int q = (int)k & 3;
    const double a = (q & 1) ? cr : sr;          // |sin x|, |cos x| up to sign
    const double b = (q & 1) ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// sin and cos to about 1e-11 absolute (mixed path only, whose outputs are FP32):
// the same reduction, then Taylor terms through x^11 and x^12 for |r| <= pi/4
// (truncation below 7e-12 and 4e-13).
__device__ __forceinline__ void sincos_reduced_short(double x, double &s, double &c)
{
    const double P1 = 0x1.921fb54442d18p+0;     // pi/2 = P1 + P2 + P3
    const double P2 = 0x1.1a62633145c07p-54;
    const double P3 = -0x1.f1976b7ed8fbcp-110;
    const double k = rint(x * 0x1.45f306dc9c883p-1);   // x * 2/pi
    double r = fma(-k, P1, x);
    r = fma(-k, P2, r);
    r = fma(-k, P3, r);
    const double r2 = r * r;
    double ps = fma_k(r2, -1.0 / 39916800.0, 1.0 / 362880.0);   // -1/11!, 1/9!
    ps = fma_k(ps, r2, -1.0 / 5040.0);
    ps = fma_k(ps, r2, 1.0 / 120.0);
    ps = fma_k(ps, r2, -1.0 / 6.0);
    const double sr = fma(r * r2, ps, r);
    double pc = fma_k(r2, 1.0 / 479001600.0, -1.0 / 3628800.0);  // 1/12!, -1/10!
    pc = fma_k(pc, r2, 1.0 / 40320.0);
    pc = fma_k(pc, r2, -1.0 / 720.0);
    pc = fma_k(pc, r2, 1.0 / 24.0);
    pc = fma(pc, r2, -0.5);
    const double cr = fma(pc, r2, 1.0);
    const int q = (int)k & 3;
    const double a = (q & 1) ? cr : sr;
    const double b = (q & 1) ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// Square root for bounds and starting values only (v_sqrt_f64, relative error
// near 2^-22): callers widen what they derive from it.
__device__ __forceinline__ double sqrt_rough(double x) { return __builtin_amdgcn_sqrt(x); }

// Trig state (cos, sin) of theta' = Theta - omega*tau kept across Newton
// updates: small changes rotate it, large ones recompute it.
struct Phase {
    double c, s;
    // from cw, sw = cos, sin(omega tau)
    __device__ __forceinline__ void set_from(const SrcRec &S, double cw, double sw)
    {
        c = S.cT * cw + S.sT * sw;      // cos(Theta - w tau)
        s = S.sT * cw - S.cT * sw;      // sin(Theta - w tau)
    }
    __device__ __forceinline__ void set(const SrcRec &S, double tau)
    {
        double sw, cw;
        sincos_reduced(S.omega * tau, sw, cw);
        set_from(S, cw, sw);
    }
    __device__ __forceinline__ void advance(const SrcRec &S, double tau_new, double dtau)
    {
        const double ang = -S.omega * dtau;    // theta' moves by -omega * dtau
        if (fabs(ang) <= 0x1p-8) {
            // |ang| <= 2^-8: Taylor through x^7 and x^6 (truncation below 5e-25)
            const double a2 = ang * ang;
            const double sa = fma(-ang * a2, fma_k(fma_k(a2, -1.0 / 5040.0, 1.0 / 120.0), -a2, 1.0 / 6.0), ang);
            const double ca = fma(a2, fma(a2, fma_k(a2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
            const double cn = c * ca - s * sa;
            const double sn = s * ca + c * sa;
            c = cn;
            s = sn;
        } else if (fabs(ang) <= 0.75) {
            double sa, ca;
            sincos_small(ang, sa, ca);
            const double cn = c * ca - s * sa;
            const double sn = s * ca + c * sa;
            c = cn;
            s = sn;
        } else {
            set(S, tau_new);
        }
    }
};

// Root bracket of g(tau) = c tau - D(tau): g < 0 below the root, g > 0 above
// (g' >= c - |v| > 0).  The ends start as geometric bounds; an end is
// "evaluated" once an iterate has landed there.
struct Bracket {
    double lo, hi;
    bool lo_ev, hi_ev;
    __device__ __forceinline__ Bracket(double l, double h) : lo(l), hi(h), lo_ev(false), hi_ev(false) {}
};

// Reciprocal for derivative terms and step sizes (v_rcp_f64 refined by one
// Newton-Raphson step): these only steer the iteration, the root itself is
// decided by g = c tau - D, which is evaluated exactly.
__device__ __forceinline__ double rcp_steer(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

// |x| and 1/|x| from s = |x|^2 (s > 0 and normal): v_rsq_f64 refined by one
// Goldschmidt step (both the root and the half-reciprocal), then Newton
// corrections of the root on its residual s - r^2.  FULL takes two corrections
// (the root to about one ulp, for the FP64 tolerance), otherwise one (relative
// error far below the 2^-32 tolerance of the mixed path).  The reciprocal keeps
// the Goldschmidt step's accuracy, which is what steering terms need.
template <bool FULL>
__device__ __forceinline__ void root_rsqrt(double s, double &r, double &ir)
{
    const double y = __builtin_amdgcn_rsq(s);
    double g = s * y, h = 0.5 * y;
    const double e = fma(-g, h, 0.5);
    g = fma(g, e, g);
    h = fma(h, e, h);
    g = fma(fma(-g, g, s), h, g);
    if (FULL) g = fma(fma(-g, g, s), h, g);
    r = g;
    ir = 2.0 * h;
}

// One safeguarded Halley update of g(tau) = c tau - D(tau) with g' = c - D'
// and g'' = -D''.  An exact root, or a step below the rounding of tau, returns
// tau itself (converged).  The Halley step is used while its denominator stays
// above g'^2 (the step is then at most twice Newton's), else Newton's.  A step
// leaving the bracket goes to the nearer end if that end has not been
// evaluated yet (the geometric bounds are often close to the root), otherwise
// bisects; so does a step onto an end already evaluated.  `free_step` reports
// whether the returned iterate is the plain Halley/Newton step (not moved onto
// the bracket).
__device__ __forceinline__ double halley_step(double tau, double D, double dD, double ddD, Bracket &b,
                                              bool &free_step)
{
    free_step = true;
    const double g = C_LIGHT * tau - D;
    if (g == 0.0) return tau;
    if (g < 0.0) {
        b.lo = tau;
        b.lo_ev = true;
    } else {
        b.hi = tau;
        b.hi_ev = true;
    }
    const double gp = C_LIGHT - dD;
    const double gp2 = gp * gp;
    const double den = fma(2.0 * gp, gp, g * ddD);          // 2 g'^2 - g g''
    // Newton's step is the same formula with the denominator 2 g'^2
    double tn = tau - 2.0 * g * gp * rcp_steer((den > gp2) ? den : 2.0 * gp2);
    if (tn == tau) return tau;
    // landing on an evaluated end again would cycle: bisect instead
    if (tn <= b.lo) {
        tn = b.lo_ev ? 0.5 * (b.lo + b.hi) : b.lo;
        free_step = false;
    } else if (tn >= b.hi) {
        tn = b.hi_ev ? 0.5 * (b.lo + b.hi) : b.hi;
        free_step = false;
    }
    return tn;
}
__device__ __forceinline__ double halley_step(double tau, double D, double dD, double ddD, Bracket &b)
{
    bool free_step;
    return halley_step(tau, D, dD, ddD, b, free_step);
}

// Plain Newton update (same safeguards), for sources whose D'' is not tracked.
__device__ __forceinline__ double newton_step(double tau, double D, double dD, Bracket &b)
{
    return halley_step(tau, D, dD, 0.0, b);
}


// Converged when the last step is below tol_rel (relative), or when both
// bracket ends have been evaluated and lie within 4 tol_rel of each other
// (rounding noise in D can make the last steps alternate around the root).
__device__ __forceinline__ bool converged(double tn, double tau, double tol_rel, const Bracket &b)
{
    return fabs(tn - tau) <= tol_rel * tn || (b.lo_ev && b.hi_ev && b.hi - b.lo <= 4.0 * tol_rel * tn);
}

// A-posteriori stop for trajectories whose g is smooth in tau (circular and
// linear oscillation, either side of the start of uniform acceleration): from
// tau, Newton's step leaves an error of about |g''| / (2 g') dtau^2 and
// Halley's a smaller (cubic) one, so once that bound is below tol/4 the new
// iterate is accepted without evaluating D at it.  Only a free (unclamped)
// step qualifies; a clamped or bisection step ends the iteration once it is
// below tol (rounding noise near the root gives free steps of a few ulp, which
// the bound accepts).
__device__ __forceinline__ bool converged_smooth(double tn, double tau, double tol_rel, const Bracket &b,
                                                 bool free_step, double dD, double ddD)
{
    const double st = tn - tau;
    return fabs(st) <= tol_rel * tn || (free_step && fabs(ddD) * (st * st) <= 0.5 * tol_rel * tn * (C_LIGHT - dD));
}

// Part of a source's retarded-time problem that does not depend on the
// observation time, for one observation point: the point in the source's frame,
// the geometric bracket on tau and the starting value with cos/sin(omega tau0).
// Field kernels build it once per (point, charge) and reuse it for every time.
struct Geo {
    double w[3];      // x - c0
    double w1, w2, w3;// circular: coordinates along e1, e2, e3; linear, accel: w1 along e1, w2 = distance^2 from the axis
    double lo, hi;    // bracket on c tau / c (circular, linear)
    double tau0;      // starting value (circular, linear)
    double cw, sw;    // cos, sin of omega tau0
    // the correction form (circular, linear; see solve_u_mixed), lengths in units of
    // D0 = c tau0: w1h = w1 / D0, w2h = w2 / D0 (circular), Ah = A / D0, kh = omega tau0,
    // K0h = (W + A^2 - D0^2) / D0^2 (circular) or (W - D0^2) / D0^2 (linear), W = |x - c0|^2
    double w1h, w2h, Ah, kh, K0h;
};

// The time-independent part of the retarded-time problem for a charge of family
// KIND (the record of any observation time), seen from x.  The stationary and
// uniform families need only w.  BRACKET: also the bracket lo, hi, which only the
// safeguarded solver reads (the correction solves' fallbacks build their own).
// The start tau0 is the RMS distance to the orbit over c: the mean of the squared
// distance lies between its least and greatest values, so the clamp to the
// bracket never moves it.  PHASE64 = false (mixed path) takes the phase of tau0
// to about 1e-11 instead of to FP64 rounding.
template <int KIND, bool BRACKET = true, bool PHASE64 = true>
__device__ __forceinline__ void geo_prepare_k(const SrcRec &S, const double x[3], Geo &g)
{
    for (int i = 0; i < 3; ++i) g.w[i] = x[i] - S.c0[i];
    if constexpr (KIND != K_CIRCULAR && KIND != K_LINEAR_OSC && KIND != K_ACCEL) return;
    const double *w = g.w;
    const double A = S.amp;
    g.w1 = w[0] * S.e1[0] + w[1] * S.e1[1] + w[2] * S.e1[2];
    if constexpr (KIND == K_CIRCULAR) {
        const double w1 = g.w1;
        const double w2 = w[0] * S.e2[0] + w[1] * S.e2[1] + w[2] * S.e2[2];
        const double w3 = w[0] * S.e3[0] + w[1] * S.e3[1] + w[2] * S.e3[2];
        g.w2 = w2;
        g.w3 = w3;
        const double WA = w1 * w1 + w2 * w2 + w3 * w3 + A * A;
        if constexpr (BRACKET) {
            const double rho = sqrt_rough(w1 * w1 + w2 * w2);
            // the distance to the orbit lies between these, so c tau does too
            // (widened by 1e-6 to cover the rough square roots)
            g.lo = sqrt_rough(w3 * w3 + (rho - A) * (rho - A)) * (INV_C * (1.0 - 1e-6));
            g.hi = sqrt_rough(w3 * w3 + (rho + A) * (rho + A)) * (INV_C * (1.0 + 1e-6));
            g.tau0 = fmin(fmax(sqrt_rough(WA) * INV_C, g.lo), g.hi);
        } else {
            g.tau0 = sqrt_rough(WA) * INV_C;
        }
        if constexpr (PHASE64) sincos_reduced(S.omega * g.tau0, g.sw, g.cw);
        else sincos_reduced_short(S.omega * g.tau0, g.sw, g.cw);
        const double D0 = C_LIGHT * g.tau0, iD0 = rcp_steer(D0);
        g.w1h = w1 * iD0;
        g.w2h = w2 * iD0;
        g.Ah = A * iD0;
        g.kh = S.omega * g.tau0;
        g.K0h = fma(-D0, D0, WA) * (iD0 * iD0);
    } else {
        const double w1 = g.w1;
        const double p0 = w[0] - w1 * S.e1[0], p1 = w[1] - w1 * S.e1[1], p2 = w[2] - w1 * S.e1[2];
        const double perp2 = p0 * p0 + p1 * p1 + p2 * p2;     // distance^2 from the axis line
        g.w2 = perp2;
        if constexpr (KIND == K_LINEAR_OSC) {
            const double W2 = perp2 + w1 * w1;
            if constexpr (BRACKET) {
                const double u = fmin(fmax(w1, -A), A);
                g.lo = sqrt_rough(perp2 + (w1 - u) * (w1 - u)) * (INV_C * (1.0 - 1e-6));
                g.hi = sqrt_rough(W2 + A * A + 2.0 * A * fabs(w1)) * (INV_C * (1.0 + 1e-6));
                g.tau0 = fmin(fmax(sqrt_rough(W2 + 0.5 * A * A) * INV_C, g.lo), g.hi);
            } else {
                g.tau0 = sqrt_rough(W2 + 0.5 * A * A) * INV_C;
            }
            if constexpr (PHASE64) sincos_reduced(S.omega * g.tau0, g.sw, g.cw);
            else sincos_reduced_short(S.omega * g.tau0, g.sw, g.cw);
            const double D0 = C_LIGHT * g.tau0, iD0 = rcp_steer(D0);
            g.w1h = w1 * iD0;
            g.w2h = 0.0;
            g.Ah = A * iD0;
            g.kh = S.omega * g.tau0;
            g.K0h = fma(-D0, D0, W2) * (iD0 * iD0);
        }
    }
}

// --- circular orbit: r = c0 + amp (cos th e1 + sin th e2), th = Theta - w tau ---
template <bool FULL>
__device__ __forceinline__ void solve_circular(const SrcRec &S, const Geo &g, int max_iter, double tol_rel, Kin &k)
{
    const double A = S.amp, om = S.omega;
    const double w1 = g.w1, w2 = g.w2, w3 = g.w3;
    Bracket b(g.lo, g.hi);
    double tau = g.tau0;
    Phase ph;
    ph.set_from(S, g.cw, g.sw);
    bool ok = (b.hi == b.lo);
    int n_it = 0;
    for (int it = 0; it < max_iter && !ok; ++it) {
        ++n_it;
        // R = x - r(t') in the orbit frame (no cancellation near the orbit)
        const double x1 = w1 - A * ph.c, x2 = w2 - A * ph.s;
        double D, iD;
        root_rsqrt<FULL>(fmax(x1 * x1 + x2 * x2 + w3 * w3, 1e-300), D, iD);
        const double Q = ph.c * x2 - ph.s * x1;              // D' = n . v = A w Q / D
        const double P = w1 * ph.c + w2 * ph.s;              // D'' = (A w^2 P - D'^2) / D
        const double dD = A * om * Q * iD;
        const double ddD = (A * om * om * P - dD * dD) * iD;
        bool free_step;
        const double tn = halley_step(tau, D, dD, ddD, b, free_step);
        ph.advance(S, tn, tn - tau);
        ok = converged_smooth(tn, tau, tol_rel, b, free_step, dD, ddD);
        tau = tn;
    }
    k.flags = ok ? 0u : FLAG_NOCONV;
    k.iters = n_it;
    k.tp = S.t - tau;
    k.cph = ph.c;
    k.sph = ph.s;
    if (FULL) {
        double ro[3], vo[3];
        for (int i = 0; i < 3; ++i) {
            ro[i] = A * (ph.c * S.e1[i] + ph.s * S.e2[i]);
            vo[i] = A * (-ph.s * S.e1[i] + ph.c * S.e2[i]);
            k.R[i] = g.w[i] - ro[i];
            k.v[i] = om * vo[i];
            k.a[i] = -om * om * ro[i];
        }
    } else {
        const float cf = (float)ph.c, sf = (float)ph.s;
        for (int i = 0; i < 3; ++i) {
            k.R[i] = g.w[i] - A * (ph.c * S.e1[i] + ph.s * S.e2[i]);
            k.bf[i] = cf * S.bw2[i] - sf * S.bw1[i];
            k.df[i] = -(cf * S.aw1[i] + sf * S.aw2[i]);
        }
    }
}

// --- linear oscillation: r = c0 + amp cos th e1 ---
template <bool FULL>
__device__ __forceinline__ void solve_linear(const SrcRec &S, const Geo &g, int max_iter, double tol_rel, Kin &k)
{
    const double A = S.amp, om = S.omega;
    const double w1 = g.w1, perp2 = g.w2;
    Bracket b(g.lo, g.hi);
    double tau = g.tau0;
    Phase ph;
    ph.set_from(S, g.cw, g.sw);
    bool ok = (b.hi == b.lo);
    int n_it = 0;
    for (int it = 0; it < max_iter && !ok; ++it) {
        ++n_it;
        const double x1 = w1 - A * ph.c;                     // R . e1
        double D, iD;
        root_rsqrt<FULL>(fmax(perp2 + x1 * x1, 1e-300), D, iD);
        const double v1 = A * om * ph.s;                     // d x1 / d tau = -v1
        const double dD = -v1 * x1 * iD;
        const double ddD = (v1 * v1 + x1 * A * om * om * ph.c - dD * dD) * iD;
        bool free_step;
        const double tn = halley_step(tau, D, dD, ddD, b, free_step);
        ph.advance(S, tn, tn - tau);
        ok = converged_smooth(tn, tau, tol_rel, b, free_step, dD, ddD);
        tau = tn;
    }
    k.flags = ok ? 0u : FLAG_NOCONV;
    k.iters = n_it;
    k.tp = S.t - tau;
    k.cph = ph.c;
    k.sph = ph.s;
    if (FULL) {
        for (int i = 0; i < 3; ++i) {
            k.R[i] = g.w[i] - A * ph.c * S.e1[i];
            k.v[i] = -A * om * ph.s * S.e1[i];
            k.a[i] = -A * om * om * ph.c * S.e1[i];
        }
    } else {
        const float cf = (float)ph.c, sf = (float)ph.s;
        for (int i = 0; i < 3; ++i) {
            k.R[i] = g.w[i] - A * ph.c * S.e1[i];
            k.bf[i] = -sf * S.bw1[i];
            k.df[i] = -cf * S.aw1[i];
        }
    }
}

// --- uniform acceleration from rest at t = 0 along e1 ---
template <bool FULL>
__device__ __forceinline__ void solve_accel(const SrcRec &S, const Geo &g, int max_iter, double tol_rel, Kin &k)
{
    const double acc = S.accel, L = S.Lmax, t = S.t;
    const double w1 = g.w1, perp2 = g.w2;
    const double W2 = perp2 + w1 * w1;
    // positions up to time t fill the segment [0, L] along e1
    const double u = fmin(fmax(w1, 0.0), L);
    const double Dnow = sqrt_rough(perp2 + (w1 - L) * (w1 - L));   // distance to the position at t
    Bracket b(sqrt_rough(perp2 + (w1 - u) * (w1 - u)) * (INV_C * (1.0 - 1e-6)),
              fmax(sqrt_rough(W2), Dnow) * (INV_C * (1.0 + 1e-6)));
    double tau = fmin(fmax(Dnow * INV_C, b.lo), b.hi);
    bool ok = (b.hi == b.lo);
    int n_it = 0;
    for (int it = 0; it < max_iter && !ok; ++it) {
        ++n_it;
        const double tp = t - tau;
        const double s = (tp > 0.0) ? 0.5 * acc * tp * tp : 0.0;   // distance along e1
        const double vel = (tp > 0.0) ? acc * tp : 0.0;
        const double x1 = w1 - s;
        double D, iD;
        root_rsqrt<FULL>(fmax(perp2 + x1 * x1, 1e-300), D, iD);
        const double dD = vel * x1 * iD;                      // d x1 / d tau = vel
        const double ddD = (vel * vel - ((tp > 0.0) ? acc * x1 : 0.0) - dD * dD) * iD;
        bool free_step;
        const double tn = halley_step(tau, D, dD, ddD, b, free_step);
        // g is smooth on either side of t' = 0 (the start of the motion), so the
        // a-posteriori stop applies to a step that stays on one side
        ok = converged_smooth(tn, tau, tol_rel, b, free_step && ((t - tn > 0.0) == (tp > 0.0)), dD, ddD);
        tau = tn;
    }
    k.flags = ok ? 0u : FLAG_NOCONV;
    k.iters = n_it;
    const double tp = t - tau;
    k.tp = tp;
    k.cph = 1.0;
    k.sph = 0.0;
    const double s = (tp >= 0.0) ? 0.5 * acc * tp * tp : 0.0;
    const double vel = (tp >= 0.0) ? acc * tp : 0.0;
    const double ac = (tp >= 0.0) ? acc : 0.0;
    for (int i = 0; i < 3; ++i) {
        k.R[i] = g.w[i] - s * S.e1[i];
        k.v[i] = vel * S.e1[i];
        k.a[i] = ac * S.e1[i];
    }
}

// --- uniform velocity: |wt + v tau| = c tau has a closed-form root ---
// FULL: correctly rounded square root and division; otherwise (the mixed path,
// whose field is FP32) the refined v_rsq_f64 root and v_rcp_f64 reciprocal,
// within a few ulp, which is all the mixed tolerance needs.
// The record holds den = c^2 - |v|^2 (amp) and its reciprocal (omega), which
// do not depend on the point.
template <bool FULL>
__device__ __forceinline__ void solve_uniform(const SrcRec &S, const double x[3], Kin &k)
{
    double wt[3];
    for (int i = 0; i < 3; ++i) wt[i] = x[i] - S.rt[i];
    const double wv = wt[0] * S.v[0] + wt[1] * S.v[1] + wt[2] * S.v[2];
    const double ww = wt[0] * wt[0] + wt[1] * wt[1] + wt[2] * wt[2];
    const double den = S.amp;
    const double disc = wv * wv + den * ww;
    double sq, isq;
    if (FULL) sq = sqrt(disc);
    else root_rsqrt<false>(fmax(disc, 1e-300), sq, isq);
    // the two algebraically equal forms, chosen to avoid cancellation
    const double tau = FULL ? ((wv >= 0.0) ? (wv + sq) / den : ww / (sq - wv))
                            : ((wv >= 0.0) ? (wv + sq) * S.omega : ww * rcp_steer(sq - wv));
    k.tp = S.t - tau;
    k.cph = 1.0;
    k.sph = 0.0;
    for (int i = 0; i < 3; ++i) {
        k.R[i] = wt[i] + S.v[i] * tau;
        k.v[i] = S.v[i];
        k.a[i] = 0.0;
    }
    k.flags = 0u;
    k.iters = 0;
}

// Mixed path, circular and linear orbits: the retarded time as a correction to
// the start, tau = tau0 (1 + u), in units of D0 = c tau0.  With the phase
// theta = theta0 - kh u (theta0 = Theta - omega tau0, kh = omega tau0), the
// condition (c tau)^2 = D^2 reads, for the circular orbit,
//   f(u) = u (2 + u) + 2 Ah P(theta) - K0h = 0,  P = w1h cos theta + w2h sin theta,
// and for the linear oscillation
//   f(u) = u (2 + u) - K0h + 2 Ah w1h cos theta - Ah^2 cos^2 theta = 0.
// f = (c tau - D)(c tau + D) / D0^2 has the root of Eq. (ret_t) as its only root
// with u > -1, needs no square root, and its terms are all of the size of
// Ah, so it is solved in FP32: Halley steps until a step is below 2^-7, the
// phase rotated from theta0 by -kh u with short Taylor polynomials (|kh u| is at
// most the charge's speed over c).  Halley's error after such a step is of the
// order of its cube, 5e-7, and FP32 rounding of f, amplified by kh, leaves the
// root's phase good to about 1e-7 rad; one Newton step in FP64 from the FP64
// phase theta0 then squares the remaining error (phase error below 1e-9 rad).
// (A stop at 2^-10 took a second FP32 step on 81 % of the benchmark's pairs for
// no change in the outputs' error; at 2^-5 the vector potential's error grew.)
// Returns false (the caller takes the safeguarded solver instead) when the FP32
// steps do not settle or leave the physical range.
__device__ __forceinline__ void rot_small_f32(float c0, float s0, float a, float &c, float &s)
{
    // sin a and cos a through a^7 and a^8: the truncation, below 2.1e-7 for
    // |a| <= 0.75 and 5.4e-9 for |a| <= 0.5, moves the FP32 root by at most
    // about Ah times that, which the FP64 Newton step that follows squares away
    const float a2 = a * a;
    const float sa = a * fmaf(a2, fmaf(a2, fmaf(a2, -1.f / 5040.f, 1.f / 120.f), -1.f / 6.f), 1.f);
    const float ca = fmaf(a2, fmaf(a2, fmaf(a2, fmaf(a2, 1.f / 40320.f, -1.f / 720.f), 1.f / 24.f), -0.5f), 1.f);
    c = c0 * ca - s0 * sa;
    s = s0 * ca + c0 * sa;
}

// The FP32 Halley steps of the correction form from u = 0, phase (c0, s0) at
// tau0: returns whether a step fell below `stop`; u and the step count n32.
template <int KIND>
__device__ __forceinline__ bool u_stage_f32(const Geo &g, double c0, double s0, float stop, float &u, int &n32)
{
    const float c0f = (float)c0, s0f = (float)s0;
    const float w1f = (float)g.w1h, w2f = (float)g.w2h, Af = (float)g.Ah, kf = (float)g.kh, K0f = (float)g.K0h;
    float c = c0f, s = s0f;
    bool ok = false;
    u = 0.f;
    n32 = 0;
    for (int it = 0; it < 4; ++it) {
        ++n32;
        float fv, fp, fpp;
        if (KIND == K_CIRCULAR) {
            const float P = fmaf(w1f, c, w2f * s), Q = fmaf(w2f, c, -w1f * s);
            fv = fmaf(u, 2.f + u, fmaf(2.f * Af, P, -K0f));
            fp = fmaf(-2.f * Af * kf, Q, 2.f + 2.f * u);
            fpp = fmaf(-2.f * Af * kf * kf, P, 2.f);
        } else {
            const float gx = fmaf(-Af, c, w1f);                  // w1h - Ah cos theta
            fv = fmaf(u, 2.f + u, fmaf(2.f * Af * w1f, c, fmaf(-Af * Af * c, c, -K0f)));
            fp = fmaf(2.f * Af * kf * s, gx, 2.f + 2.f * u);
            fpp = fmaf(-2.f * Af * kf * kf, fmaf(c, gx, -Af * s * s), 2.f);
        }
        const float fp2 = fp * fp;
        float den = fmaf(2.f, fp2, -fv * fpp);
        den = den > fp2 ? den : 2.f * fp2;
        const float d = -2.f * fv * fp * __builtin_amdgcn_rcpf(den);
        u += d;
        if (fabsf(d) <= stop) {
            ok = true;
            break;
        }
        rot_small_f32(c0f, s0f, -kf * u, c, s);
    }
    return ok;
}

// (cos, sin) of the phase theta0 - kh u: (c0, s0) rotated by a = -kh u, |a| <= 0.75,
// through a^11 and a^12 (truncation below 2e-17).
__device__ __forceinline__ void rot_phase(double c0, double s0, double a, double &c, double &s)
{
    const double a2 = a * a;
    const double sa = a * fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, -1.0 / 39916800.0, 1.0 / 362880.0),
                                                          -1.0 / 5040.0), 1.0 / 120.0), -1.0 / 6.0), 1.0);
    const double ca = fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, 1.0 / 479001600.0, -1.0 / 3628800.0),
                                                                   1.0 / 40320.0), -1.0 / 720.0), 1.0 / 24.0), -0.5), 1.0);
    c = c0 * ca - s0 * sa;
    s = s0 * ca + c0 * sa;
}

// The same rotation for the mixed path, through a^9 and a^10 (truncation below
// 1.1e-9 for |a| <= 0.75 and 1.3e-11 for |a| <= 0.5, against FP32 outputs).
__device__ __forceinline__ void rot_phase_short(double c0, double s0, double a, double &c, double &s)
{
    const double a2 = a * a;
    const double sa = a * fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, 1.0 / 362880.0, -1.0 / 5040.0), 1.0 / 120.0),
                                          -1.0 / 6.0), 1.0);
    const double ca = fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, fma_k(a2, -1.0 / 3628800.0, 1.0 / 40320.0),
                                                          -1.0 / 720.0), 1.0 / 24.0), -0.5), 1.0);
    c = c0 * ca - s0 * sa;
    s = s0 * ca + c0 * sa;
}

// f(u) and f'(u) of the correction form in FP64 at phase (cd, sd).
template <int KIND>
__device__ __forceinline__ void u_f64(const Geo &g, double ud, double cd, double sd, double &fv, double &fp)
{
    if (KIND == K_CIRCULAR) {
        const double P = fma(g.w1h, cd, g.w2h * sd), Q = fma(g.w2h, cd, -g.w1h * sd);
        fv = fma(ud, 2.0 + ud, fma(2.0 * g.Ah, P, -g.K0h));
        fp = fma(-2.0 * g.Ah * g.kh, Q, 2.0 + 2.0 * ud);
    } else {
        const double gx = fma(-g.Ah, cd, g.w1h);
        fv = fma(ud, 2.0 + ud, fma(2.0 * g.Ah * g.w1h, cd, fma(-g.Ah * g.Ah * cd, cd, -g.K0h)));
        fp = fma(2.0 * g.Ah * g.kh * sd, gx, 2.0 + 2.0 * ud);
    }
}

template <int KIND>
__device__ __forceinline__ bool solve_u_mixed(const SrcRec &S, const Geo &g, Kin &k)
{
    // phase at tau0 for this observation time (FP64)
    const double c0 = S.cT * g.cw + S.sT * g.sw;
    const double s0 = S.sT * g.cw - S.cT * g.sw;
    float u;
    int n32;
    const bool ok = u_stage_f32<KIND>(g, c0, s0, 0x1p-7f, u, n32);
    const double a = -g.kh * (double)u;
    if (!ok || !(fabs(a) <= 0.75) || !(u > -0.5f)) return false;
    // one Newton step in FP64 from the exact phase (f' in FP64 too: an FP32 f' + f'' d
    // from the last Halley step was tried, and where the terms of f' cancel its
    // rounding left the vector potential's pointwise error 30 times larger)
    double cd, sd;
    rot_phase_short(c0, s0, a, cd, sd);
    double ud = (double)u, fv, fp;
    u_f64<KIND>(g, ud, cd, sd, fv, fp);
    // v_rcp_f64 unrefined (relative error below 2^-26): the step is of the size
    // of the FP32 stage's remaining error, so this moves u by far less than 1e-13
    const double du = -fv * __builtin_amdgcn_rcp(fp);
    ud += du;
    // rotate the phase by the correction's angle e (second order: |e| is of the
    // order of kh times the FP32 steps' error, so e^3 / 6 stays far below FP32
    // resolution)
    const double e = -g.kh * du, ce = fma(-0.5 * e, e, 1.0);
    const double cn = cd * ce - sd * e, sn = sd * ce + cd * e;
    const double tau = fma(g.tau0, ud, g.tau0);
    k.flags = 0u;
    k.iters = n32 + 1;
    k.tp = S.t - tau;
    k.cph = cn;
    k.sph = sn;
    const double A = S.amp;
    const float cf = (float)cn, sf = (float)sn;
    if (KIND == K_CIRCULAR) {
        for (int i = 0; i < 3; ++i) {
            k.R[i] = g.w[i] - A * (cn * S.e1[i] + sn * S.e2[i]);
            k.bf[i] = cf * S.bw2[i] - sf * S.bw1[i];
            k.df[i] = -(cf * S.aw1[i] + sf * S.aw2[i]);
        }
    } else {
        for (int i = 0; i < 3; ++i) {
            k.R[i] = g.w[i] - A * cn * S.e1[i];
            k.bf[i] = -sf * S.bw1[i];
            k.df[i] = -cf * S.aw1[i];
        }
    }
    return true;
}

// FP64 path, circular and linear orbits: the correction form with the FP32
// steps above, then two Newton steps in FP64 (the first from the exact phase
// rotated by the polynomial, the second from a fourth-order rotation by the
// first step's angle e: the truncation e^5 / 120 is below 1e-17 for |e| <= 1e-3,
// and a larger angle sends the point to the safeguarded solver).  Newton squares
// the error, so the FP32 steps' remaining error (about their last step cubed,
// and a phase error of about 1e-7 rad from FP32 rounding) is at rounding level
// after the second step.  The root is accepted when Newton's bound on the remaining error,
// |f''| du^2 / (2 |f'|) with |f''| <= 2 + 2 Ah kh^2 M (M = |(w1h, w2h)| for the
// circular orbit, |w1h| + Ah for the linear one), is below 2^-54, about half an
// ulp of u near 1, and the second step's angle is below 2^-27 (its phase follows
// by a first-order rotation); otherwise (and when the FP32 steps do not settle)
// the caller takes the safeguarded Halley solver.  R, v and a come out in FP64.
template <int KIND>
__device__ __forceinline__ bool solve_u_full(const SrcRec &S, const Geo &g, Kin &k)
{
    const double c0 = S.cT * g.cw + S.sT * g.sw;
    const double s0 = S.sT * g.cw - S.cT * g.sw;
    float u;
    int n32;
    // the FP32 steps run to 2^-10 here (two FP64 Newton steps then meet the 2^-54
    // bound below; from 2^-7 more points missed it and took the safeguarded solver)
    const bool ok = u_stage_f32<KIND>(g, c0, s0, 0x1p-10f, u, n32);
    const double a = -g.kh * (double)u;
    if (!ok || !(fabs(a) <= 0.75) || !(u > -0.5f)) return false;
    double cd, sd;
    rot_phase(c0, s0, a, cd, sd);
    double ud = (double)u, fv, fp;
    // first step: the phase follows by a fourth-order rotation (its angle is below
    // 1e-3 on acceptance, so the truncation e^5 / 120 is below 1e-17)
    u_f64<KIND>(g, ud, cd, sd, fv, fp);
    double du = -fv * rcp_steer(fp);
    ud += du;
    double e = -g.kh * du;
    bool small = fabs(e) <= 1e-3;
    {
        const double e2 = e * e;
        const double ce = fma(e2, fma(e2, 1.0 / 24.0, -0.5), 1.0), se = e * fma(e2, -1.0 / 6.0, 1.0);
        const double cn = cd * ce - sd * se, sn = sd * ce + cd * se;
        cd = cn;
        sd = sn;
    }
    // second step: its angle is below 2^-27 on acceptance, so a first-order
    // rotation is exact to e^2 / 2 < 3e-17
    u_f64<KIND>(g, ud, cd, sd, fv, fp);
    du = -fv * rcp_steer(fp);
    ud += du;
    e = -g.kh * du;
    small = small && fabs(e) <= 0x1p-27;
    {
        const double cn = fma(-sd, e, cd), sn = fma(cd, e, sd);
        cd = cn;
        sd = sn;
    }
    const double M = KIND == K_CIRCULAR ? sqrt_rough(fma(g.w1h, g.w1h, g.w2h * g.w2h)) * (1.0 + 1e-6)
                                        : fabs(g.w1h) + g.Ah;
    const double f2 = fma(2.0 * g.Ah * g.kh * g.kh, M, 2.0);
    if (!small || !(ud > -0.5) || !(f2 * du * du <= 0x1p-53 * fabs(fp))) return false;
    const double tau = fma(g.tau0, ud, g.tau0);
    k.flags = 0u;
    k.iters = n32 + 2;
    k.tp = S.t - tau;
    k.cph = cd;
    k.sph = sd;
    const double A = S.amp, om = S.omega;
    for (int i = 0; i < 3; ++i) {
        if (KIND == K_CIRCULAR) {
            const double ro = A * (cd * S.e1[i] + sd * S.e2[i]);
            k.R[i] = g.w[i] - ro;
            k.v[i] = om * A * (-sd * S.e1[i] + cd * S.e2[i]);
            k.a[i] = -om * om * ro;
        } else {
            k.R[i] = g.w[i] - A * cd * S.e1[i];
            k.v[i] = -A * om * sd * S.e1[i];
            k.a[i] = -A * om * om * cd * S.e1[i];
        }
    }
    return true;
}

// Mixed path, uniform acceleration from rest: the same correction form,
// tau = tau0 (1 + u) with tau0 = D0 / c the light time from the charge's
// position at t (distance D0).  With L = a t^2 / 2 travelled by t and
//   m = a tau (2t - tau) / 2   (tau <= t),   m = L   (tau > t, before the start),
// the charge sits at L - m along e1 at t - tau, so with X = w1 - L
//   f(u) = u (2 + u) - mh (2 Xh + mh) - K0h,  mh = m / D0 = (a / 2c)(1 + u)(2t - tau),
// K0h = (perp^2 + X^2 - D0^2) / D0^2, where m and its first derivative are
// continuous at the start of the motion.  FP32 Halley steps, then one FP64
// Newton step, as for the oscillating families.  f has one root with u > -1
// and f' > 0 around it (f' = 2 (c^2 tau - x1 v) / (c tau0)^2 with |x1 v| < c D),
// so a lane whose FP32 steps did not settle continues with FP64 Newton steps
// (up to 30) instead of a separate bracketed solver, whose registers would
// spill the kernel; only if those fail too is the point flagged.
// FULL (the FP64 path): the FP32 steps run to 2^-10 and the FP64 Newton steps
// continue until a step is below 2^-50 (1 + |u|), three in the usual case (the
// second leaves about the square of the FP32 stage's error, the third confirms);
// returns false if they do not, and the caller takes the safeguarded solver.
template <bool FULL = false>
__device__ __forceinline__ bool solve_u_accel(const SrcRec &S, const Geo &g, Kin &k)
{
    const double t = S.t, acc = S.accel, L = S.Lmax;
    const double X = g.w1 - L;
    const double Dn2 = fma(X, X, g.w2);
    const double D0 = sqrt_rough(Dn2);
    if (!(D0 > 0.0)) return false;
    const double iD0 = rcp_steer(D0), tau0 = D0 * INV_C;
    const double Xh = X * iD0, K0h = fma(-D0, D0, Dn2) * (iD0 * iD0), gh = acc * (0.5 * INV_C), Lh = L * iD0;
    const float Xf = (float)Xh, K0f = (float)K0h, gf = (float)gh, Lf = (float)Lh, tf = (float)t, t0f = (float)tau0;
    float u = 0.f;
    bool ok = false;
    int n_it = 0;
    for (int it = 0; it < 6; ++it) {
        ++n_it;
        const float tau = fmaf(t0f, u, t0f);
        const bool moving = tau < tf;
        const float m = moving ? gf * (1.f + u) * (2.f * tf - tau) : Lf;
        const float mp = moving ? 2.f * gf * (tf - tau) : 0.f;
        const float mpp = moving ? -2.f * gf * t0f : 0.f;
        const float xm = Xf + m;
        const float fv = fmaf(u, 2.f + u, fmaf(-m, Xf + xm, -K0f));
        const float fp = fmaf(-2.f * mp, xm, 2.f + 2.f * u);
        const float fpp = fmaf(-2.f, fmaf(mpp, xm, mp * mp), 2.f);
        const float fp2 = fp * fp;
        float den = fmaf(2.f, fp2, -fv * fpp);
        den = den > fp2 ? den : 2.f * fp2;
        const float d = -2.f * fv * fp * __builtin_amdgcn_rcpf(den);
        u += d;
        if (fabsf(d) <= (FULL ? 0x1p-10f : 0x1p-7f)) {
            ok = true;
            break;
        }
    }
    // FP64 Newton: one step after settled FP32 steps (FULL: until converged, at most
    // three), else until it settles
    double ud = (ok && u > -0.5f) ? (double)u : 0.0;
    const int n_newton = (ok && u > -0.5f) ? (FULL ? 3 : 1) : 30;
    bool conv = !FULL && n_newton == 1;
    for (int it = 0; it < n_newton; ++it) {
        ++n_it;
        const double tau = fma(tau0, ud, tau0);
        const bool moving = tau < t;
        const double m = moving ? gh * (1.0 + ud) * (2.0 * t - tau) : Lh;
        const double mp = moving ? 2.0 * gh * (t - tau) : 0.0;
        const double xm = Xh + m;
        const double fv = fma(ud, 2.0 + ud, fma(-m, Xh + xm, -K0h));
        const double fp = fma(-2.0 * mp, xm, 2.0 + 2.0 * ud);
        const double du = -fv * rcp_steer(fp);
        ud += du;
        if (!conv && fabs(du) <= 0x1p-50 * (1.0 + fabs(ud))) {
            conv = true;
            break;
        }
    }
    if (!(ud > -0.5)) conv = false;
    const double tau = fma(tau0, ud, tau0);
    const double tp = t - tau;
    const double sd = (tp > 0.0) ? 0.5 * acc * tp * tp : 0.0;
    const double vel = (tp > 0.0) ? acc * tp : 0.0;
    const double ac = (tp > 0.0) ? acc : 0.0;
    k.flags = conv ? 0u : FLAG_NOCONV;
    k.iters = n_it;
    k.tp = tp;
    k.cph = 1.0;
    k.sph = 0.0;
    for (int i = 0; i < 3; ++i) {
        k.R[i] = g.w[i] - sd * S.e1[i];
        k.v[i] = vel * S.e1[i];
        k.a[i] = ac * S.e1[i];
    }
    return conv;
}

// The rare fallback of the correction solves for the oscillating families (a
// solve that did not settle): the safeguarded solver on a geometry rebuilt here
// with its bracket, so that the main path neither builds the bracket nor keeps
// the frame coordinates live across the times.
template <bool FULL, int KIND>
__device__ __forceinline__ void retarded_fallback(const SrcRec &S, const double x[3], int max_iter, double tol_rel,
                                                  Kin &k)
{
    Geo gf;
    geo_prepare_k<KIND>(S, x, gf);
    if constexpr (KIND == K_CIRCULAR) solve_circular<FULL>(S, gf, max_iter, tol_rel, k);
    else solve_linear<FULL>(S, gf, max_iter, tol_rel, k);
}

// Retarded kinematics of a source S of family KIND (its record for the
// observation time) seen from point x, with g = geo_prepare_k<KIND, BRACKET,
// PHASE64>(record of any time of this source, x).  FULL: FP64 tolerance (square
// roots to about one ulp); otherwise the mixed path's relaxed tolerance.
// CORR (FULL only): the correction solves first, their fallback on a rebuilt
// geometry (g needs no bracket); without it the safeguarded Halley solvers on g
// directly (g with its bracket; fewer live registers, for kernels whose occupancy
// the correction solve would cost).  The mixed path (FULL = false) always takes
// the correction solves, with PHASE64 = false allowed.
template <bool FULL, bool CORR, int KIND>
__device__ __forceinline__ void retarded_kind(const SrcRec &S, const Geo &g, const double x[3], int max_iter,
                                              double tol_rel, Kin &k)
{
    if constexpr (KIND == K_CIRCULAR || KIND == K_LINEAR_OSC) {
        if (FULL && !CORR) {
            if constexpr (KIND == K_CIRCULAR) solve_circular<true>(S, g, max_iter, tol_rel, k);
            else solve_linear<true>(S, g, max_iter, tol_rel, k);
        } else if (FULL) {
            if (!solve_u_full<KIND>(S, g, k)) retarded_fallback<true, KIND>(S, x, max_iter, tol_rel, k);
        } else if (!solve_u_mixed<KIND>(S, g, k)) {
            retarded_fallback<false, KIND>(S, x, max_iter, tol_rel, k);
            k.iters |= ITER_FALLBACK;
        }
    } else if constexpr (KIND == K_ACCEL) {
        if (FULL) {
            if (!CORR || !solve_u_accel<true>(S, g, k)) solve_accel<FULL>(S, g, max_iter, tol_rel, k);
        } else {
            solve_u_accel(S, g, k);
            kin_beta_from_va(k);
        }
    } else if constexpr (KIND == K_UNIFORM_VELOCITY) {
        solve_uniform<FULL>(S, x, k);
        if (!FULL)
            for (int i = 0; i < 3; ++i) {     // kin_beta_from_va's values, from the record
                k.bf[i] = S.bw1[i];
                k.df[i] = 0.f;
            }
    } else {
        for (int i = 0; i < 3; ++i) { k.R[i] = g.w[i]; k.v[i] = 0.0; k.a[i] = 0.0; k.bf[i] = 0.f; k.df[i] = 0.f; }
        k.tp = S.t - sqrt(g.w[0] * g.w[0] + g.w[1] * g.w[1] + g.w[2] * g.w[2]) * INV_C;
        k.cph = 1.0;
        k.sph = 0.0;
        k.flags = 0u;
        k.iters = 0;
    }
}

template <typename F> __device__ __forceinline__ F recip(F x);
template <> __device__ __forceinline__ float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }
// FP64: v_rcp_f64 and two Newton-Raphson steps (within about one ulp)
template <> __device__ __forceinline__ double recip<double>(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// Lienard-Wiechert outputs of one charge from its retarded kinematics, in
// precision F: out = (Phi, A, E, B).  With u = n - beta and kappa = 1 - n.beta,
// the radiation term's double cross product expands (BAC-CAB, n.u = kappa) to
//   n x (u x beta_dot) = u (n . beta_dot) - kappa beta_dot,
// so E = kq / (kappa^3 R) [u ((1 - beta^2)/R + n.beta_dot / c) - kappa beta_dot / c]
// for the total field (Eq. (E)); the Coulomb and radiation parts keep their
// own terms.  B = n x E / c (Eq. (B)), Phi = kq / (kappa R) (Eq. (V)),
// A = Phi beta / c (Eq. (A) in SI form).
// |R| and 1/|R| in precision F: FP32 through v_rsq_f32; FP64 from the refined
// v_rsq_f64 with one more Newton-Raphson step on the reciprocal (both within
// about one ulp).  |R| = 0 gives NaN, which the caller masks.
__device__ __forceinline__ void dist_inv(float R0, float R1, float R2, float &D, float &iD)
{
    const float D2 = R0 * R0 + R1 * R1 + R2 * R2;
    iD = __builtin_amdgcn_rsqf(D2);
    D = D2 * iD;
}
__device__ __forceinline__ void dist_inv(double R0, double R1, double R2, double &D, double &iD)
{
    root_rsqrt<true>(R0 * R0 + R1 * R1 + R2 * R2, D, iD);
    iD = fma(iD, fma(-D, iD, 1.0), iD);
}

// Returns the retarded distance |R| in precision F (for masking).  IC = false
// leaves out the factor 1/c of A and B (out[1..3] = Phi beta, out[7..9] = n x E),
// for callers that sum over charges first and scale the sums once.
template <typename F, bool IC = true>
__device__ __forceinline__ F lw_terms(const Kin &k, F kq, int field_kind, F out[10])
{
    const F R0 = (F)k.R[0], R1 = (F)k.R[1], R2 = (F)k.R[2];
    F D, iD;
    dist_inv(R0, R1, R2, D, iD);
    const F n0 = R0 * iD, n1 = R1 * iD, n2 = R2 * iD;
    F b0, b1, b2, d0, d1, d2;
    if constexpr (sizeof(F) == 4) {
        b0 = k.bf[0]; b1 = k.bf[1]; b2 = k.bf[2];
        d0 = k.df[0]; d1 = k.df[1]; d2 = k.df[2];
    } else {
        b0 = k.v[0] * INV_C; b1 = k.v[1] * INV_C; b2 = k.v[2] * INV_C;
        d0 = k.a[0] * INV_C; d1 = k.a[1] * INV_C; d2 = k.a[2] * INV_C;
    }
    const F ic = (F)INV_C;
    const F nb = n0 * b0 + n1 * b1 + n2 * b2;
    const F kappa = (F)1 - nb;
    const F bb = b0 * b0 + b1 * b1 + b2 * b2;
    const F u0 = n0 - b0, u1 = n1 - b1, u2 = n2 - b2;
    const F nd = n0 * d0 + n1 * d1 + n2 * d2;
    const F ik = recip<F>(kappa);
    const F kqD = kq * iD;
    const F phi = kqD * ik;
    const F f = phi * ik * ik;                              // kq / (kappa^3 R)
    F cu, cd;                                               // E = f (u cu - beta_dot cd)
    if (field_kind == F_COULOMB) {
        cu = ((F)1 - bb) * iD;
        cd = (F)0;
    } else if (field_kind == F_RADIATION) {
        cu = nd * ic;
        cd = kappa * ic;
    } else {
        cu = ((F)1 - bb) * iD + nd * ic;
        cd = kappa * ic;
    }
    const F E0 = f * (u0 * cu - d0 * cd);
    const F E1 = f * (u1 * cu - d1 * cd);
    const F E2 = f * (u2 * cu - d2 * cd);
    const F m0 = IC ? n0 * ic : n0, m1 = IC ? n1 * ic : n1, m2 = IC ? n2 * ic : n2;  // n / c
    const F pc = IC ? phi * ic : phi;
    out[0] = phi;
    out[1] = pc * b0;
    out[2] = pc * b1;
    out[3] = pc * b2;
    out[4] = E0;
    out[5] = E1;
    out[6] = E2;
    out[7] = m1 * E2 - m2 * E1;
    out[8] = m2 * E0 - m0 * E2;
    out[9] = m0 * E1 - m1 * E0;
    return D;
}

// Reverse of lw_terms<double>: given the cotangent ob of (Phi, A, E, B), the
// cotangents of R, v, a and of kq = q / (4 pi eps0).  EONLY: only E has a
// cotangent (ob[4..6]; the other entries are not read), as for objectives of
// |E|^2.  The reverses of Phi, A and B are then left out, which gives the
// values of the general form with zero cotangents there (it adds only zeros).
// FAST: 1/|R| and 1/kappa from the refined hardware reciprocal square root and
// reciprocal (within an ulp or two) instead of the correctly rounded square
// root and divisions, as the forward FP64 evaluator takes them.
template <bool EONLY = false, bool FAST = false>
__device__ __forceinline__ void lw_terms_vjp(const Kin &k, double kq, int field_kind, const double ob[10],
                                             double Rb[3], double vb[3], double ab[3], double &kqb, double n[3],
                                             double &kappa_out)
{
    const double ic = INV_C;
    double D, iD;
    if constexpr (FAST) {
        dist_inv(k.R[0], k.R[1], k.R[2], D, iD);
    } else {
        D = sqrt(k.R[0] * k.R[0] + k.R[1] * k.R[1] + k.R[2] * k.R[2]);
        iD = 1.0 / D;
    }
    double b[3], d[3], u[3];
    for (int i = 0; i < 3; ++i) {
        n[i] = k.R[i] * iD;
        b[i] = k.v[i] * ic;
        d[i] = k.a[i] * ic;
        u[i] = n[i] - b[i];
    }
    const double nb = n[0] * b[0] + n[1] * b[1] + n[2] * b[2];
    const double kappa = 1.0 - nb;
    const double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    const double ik = FAST ? recip<double>(kappa) : 1.0 / kappa;
    const double kqD = kq * iD;
    const double phi = kqD * ik;
    const double f = phi * ik * ik;
    const bool coul = field_kind != F_RADIATION, rad = field_kind != F_COULOMB;
    const double cu = (coul ? (1.0 - bb) * iD : 0.0) + (rad ? nd * ic : 0.0);
    const double cd = rad ? kappa * ic : 0.0;
    double W[3], E[3], m[3];
    for (int i = 0; i < 3; ++i) {
        W[i] = u[i] * cu - d[i] * cd;
        E[i] = f * W[i];
        m[i] = n[i] * ic;
    }
    const double pc = phi * ic;
    // ---- reverse ----
    const double Eb[3] = {ob[4], ob[5], ob[6]};
    double mb[3] = {0.0, 0.0, 0.0}, Et[3] = {Eb[0], Eb[1], Eb[2]};
    double Phib = 0.0, pcb = 0.0, bbar[3] = {0.0, 0.0, 0.0};
    if constexpr (!EONLY) {
        Phib = ob[0];
        const double Ab[3] = {ob[1], ob[2], ob[3]};
        const double Bb[3] = {ob[7], ob[8], ob[9]};
        // B = m x E
        mb[0] = E[1] * Bb[2] - E[2] * Bb[1];
        mb[1] = E[2] * Bb[0] - E[0] * Bb[2];
        mb[2] = E[0] * Bb[1] - E[1] * Bb[0];
        Et[0] = Eb[0] + (Bb[1] * m[2] - Bb[2] * m[1]);
        Et[1] = Eb[1] + (Bb[2] * m[0] - Bb[0] * m[2]);
        Et[2] = Eb[2] + (Bb[0] * m[1] - Bb[1] * m[0]);
        // A = pc b
        pcb = Ab[0] * b[0] + Ab[1] * b[1] + Ab[2] * b[2];
        for (int i = 0; i < 3; ++i) bbar[i] = pc * Ab[i];
    }
    // E = f W, W = u cu - d cd
    const double fb = Et[0] * W[0] + Et[1] * W[1] + Et[2] * W[2];
    double ub[3], dbar[3];
    double cub = 0.0, cdb = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double Wb = f * Et[i];
        ub[i] = Wb * cu;
        cub += Wb * u[i];
        dbar[i] = -Wb * cd;
        cdb -= Wb * d[i];
    }
    // phi = kqD ik feeds Phi, pc and f
    const double phib = EONLY ? fb * ik * ik : Phib + pcb * ic + fb * ik * ik;
    const double ikb_f = fb * 2.0 * phi * ik;
    double ikb = ikb_f + phib * kqD;
    const double kqDb = phib * ik;
    // cu, cd
    const double bbb = coul ? -cub * iD : 0.0;
    double iDb = coul ? cub * (1.0 - bb) : 0.0;
    const double ndb = rad ? cub * ic : 0.0;
    double kappab = rad ? cdb * ic : 0.0;
    // m = n / c
    double nbar[3] = {0.0, 0.0, 0.0};
    if constexpr (!EONLY)
        for (int i = 0; i < 3; ++i) nbar[i] = mb[i] * ic;
    // kqD = kq iD
    iDb += kqDb * kq;
    kqb = kqDb * iD;
    // ik = 1 / kappa
    kappab -= ikb * ik * ik;
    // nd = n . d
    for (int i = 0; i < 3; ++i) {
        nbar[i] += ndb * d[i] + ub[i];
        dbar[i] += ndb * n[i];
        bbar[i] += -ub[i] + 2.0 * bbb * b[i];
    }
    // kappa = 1 - n . b
    const double nbb = -kappab;
    for (int i = 0; i < 3; ++i) {
        nbar[i] += nbb * b[i];
        bbar[i] += nbb * n[i];
        vb[i] = bbar[i] * ic;
        ab[i] = dbar[i] * ic;
    }
    // n = R iD with iD = 1/|R|
    iDb += nbar[0] * k.R[0] + nbar[1] * k.R[1] + nbar[2] * k.R[2];
    const double s = -iDb * iD * iD;
    for (int i = 0; i < 3; ++i) Rb[i] = nbar[i] * iD + s * n[i];
    kappa_out = kappa;
}

}  // namespace lw

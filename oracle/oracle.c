/*
 * Plain FP64 CPU oracle for the phase-space hot path of MadSpace
 * (Heimel, Mattelaer, Winterhalder, arXiv:2602.06895).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library.  It shares no
 * code with the HIP library: different sources, headers and channel compiler.
 *
 * Every function follows the paper's definitions step by step, in FP64,
 * without blocking, fusion or reordering; events are independent and are
 * distributed over OpenMP threads with a static schedule.
 *
 * Conventions: metric (+,-,-,-), p = (E, px, py, pz), GeV.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* Perturbation builds (forward-error estimation only, never the reference):
 * with ORC_LIBM_NUDGE = +1 or -1 every transcendental and square-root result
 * is moved by one ulp up or down, standing in for a different math library or
 * a different rounding of its argument.  The exact results 0 and +-1 are left
 * alone (every library returns them exactly). */
#ifdef ORC_LIBM_NUDGE
static double orc_nudge(double v)
{
    if (v == 0.0 || v == 1.0 || v == -1.0 || !isfinite(v)) return v;
    return nextafter(v, ORC_LIBM_NUDGE > 0 ? INFINITY : -INFINITY);
}
#define pow(a, b) orc_nudge(pow(a, b))
#define exp(a) orc_nudge(exp(a))
#define log(a) orc_nudge(log(a))
#define sqrt(a) orc_nudge(sqrt(a))
#define atan(a) orc_nudge(atan(a))
#define tan(a) orc_nudge(tan(a))
#define sin(a) orc_nudge(sin(a))
#define cos(a) orc_nudge(cos(a))
#define atan2(a, b) orc_nudge(atan2(a, b))
#define cosh(a) orc_nudge(cosh(a))
#define sinh(a) orc_nudge(sinh(a))
#define asinh(a) orc_nudge(asinh(a))
#endif

/* Planted mistakes (pin-strength tests only, never the reference): a build
 * with ORC_MUTATE = k carries mistake k, which some pin must detect:
 *   1  the toy PDF's (1 - x) exponent off by one
 *   2  mu instead of mu^2 in the massless propagator factor
 *   3  q = p_a + sum p_k for a t-type propagator (wrong sign convention)
 *   4  the Breit-Wigner factor with Gamma^2 in place of M^2 Gamma^2 */
#ifndef ORC_MUTATE
#define ORC_MUTATE 0
#endif

#define ORC_MAX_NODES 64
#define ORC_MAX_FINAL 16
#define ORC_MAX_DIMS 64
/* Recovered uniforms farther than this outside [0, 1] mark an event that is
 * not in the channel's image (its density there is 0). */
#define ORC_SUPPORT_MARGIN 1e-6
#define ORC_MAX_PROPS 64

enum { ORC_LEAF = 0, ORC_CLUSTER = 1, ORC_TNODE = 2 };

/* One channel = one diagram topology.  The root node is sampled first: its
 * invariant is s-hat.  For a t-channel topology the root is the effective
 * t-node whose children are the legs along the spine from a to b (section
 * "s-channel integration order": the t-channel part is one node with
 * kappa+1 children); for a pure s-channel topology it is the cluster that
 * decays at s-hat. */
typedef struct {
    int32_t n_nodes, root, n_sorder, n_dec;
    const int32_t* kind;        /* [n_nodes] */
    const int32_t* particle;    /* leaf: final-state index 0..n-1 */
    const int32_t* parent;      /* -1 for the root */
    const int32_t* child_start; /* index into children[] */
    const int32_t* child_count;
    const int32_t* children;
    const double* mass;         /* leaf mass, or propagator mass of a cluster */
    const double* width;        /* propagator width (clusters) */
    const double* nu;           /* power-law exponent per cluster (or default) */
    const char* t_order;        /* kappa-1 letters 'A'/'B' */
    const int32_t* s_order;     /* clusters other than the root, sampling order */
    const int32_t* dec_order;   /* clusters decayed with (phi,theta), parents first */
    const int32_t* rambo;       /* FastRambo cluster: its particle count - 1 (k), else 0 */
    int32_t chili;              /* 1: a Chili channel (no tree) */
    int32_t st;                 /* 1: t-chain blocks with a recoil use (s~, t) */
} orc_channel;

typedef struct {
    int32_t hadronic;   /* 1: PDF convolution with s-hat sampling; 0: fixed sqrt(s) */
    int32_t n_final;
    double s_lab;
    double shat_min;
    double nu;          /* default power-law exponent */
    double reg_a;       /* auxiliary negative mass parameter m^2 = -a */
    const double* mass; /* [n_final] */
    /* integrand */
    int32_t pdf;
    double pdf_a, pdf_b;
    double pt_min;      /* <= 0: no cut */
    int32_t ang;        /* -1, or particle index k: f *= 1 + cos^2(theta_k) */
    int32_t n_prop;
    const int32_t* prop_t;    /* 1: q = p_a - sum p_k;  0: q = sum p_k */
    const uint32_t* prop_set; /* bit k -> final-state particle k */
    const int32_t* prop_bw;   /* 1: 1/((q^2-M^2)^2 + M^2 G^2);  0: 1/(|q^2| + mu^2) */
    const double* prop_m;
    const double* prop_w;
    const double* prop_mu;
    /* channel weights alpha_c(x): every channel's propagator list */
    int32_t n_chan;
    double alpha_mu;
    const int32_t* ch_start;  /* [n_chan + 1] into chp_* */
    const int32_t* chp_t;
    const uint32_t* chp_set;
    const double* chp_m;
    const double* chp_w;
    /* 1 for a channel without a diagram (Chili): constant share 1 / n_chan */
    const int32_t* ch_prior;
} orc_process;

/* ------------------------------------------------------------------------ */
/* Elementary pieces                                                         */
/* ------------------------------------------------------------------------ */

static const double ORC_PI = 3.14159265358979323846;

/* Kallen function lambda(x, y, z) = (x - y - z)^2 - 4 y z (section 2.2.3). */
double orc_kallen(double x, double y, double z)
{
    double d = x - y - z;
    return d * d - 4.0 * y * z;
}

static double mdot(const double a[4], const double b[4])
{
    return a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
}

/* Power-law invariant mapping G_nu with its Jacobian 1/g (equations
 * prop_stable_nu, prop_stable_nu1 for nu = 1, prop_flat for nu = 0). */
double orc_map_nu(double r, double m2, double nu, double xmin, double xmax, double* jac)
{
    if (nu == 0.0) {
        *jac = xmax - xmin;
        return xmin + (xmax - xmin) * r;
    }
    if (nu == 1.0) {
        double lmax = log(xmax - m2), lmin = log(xmin - m2);
        double x = exp(r * lmax + (1.0 - r) * lmin) + m2;
        *jac = (x - m2) * (lmax - lmin);
        return x;
    }
    double e = 1.0 - nu;
    double A = pow(xmax - m2, e), B = pow(xmin - m2, e);
    double x = pow(r * A + (1.0 - r) * B, 1.0 / e) + m2;
    *jac = (A - B) * pow(x - m2, nu) / e;
    return x;
}

/* Breit-Wigner mapping G_BW with its Jacobian 1/g (equation prop_massive). */
double orc_map_bw(double r, double m, double w, double xmin, double xmax, double* jac)
{
    double m2 = m * m, mw = m * w;
    double u1 = atan((xmin - m2) / mw), u2 = atan((xmax - m2) / mw);
    double x = mw * tan(u1 + (u2 - u1) * r) + m2;
    *jac = (u2 - u1) * ((x - m2) * (x - m2) + mw * mw) / mw;
    return x;
}

/* FastRambo (section 2.2.9).  The single-bin rational-quadratic function
 * with slope c at y = 0 and slope 0 at y = 1, and its closed-form inverse. */
double orc_rqf(double y, double c)
{
    return (y * y + c * y * (1.0 - y)) / (1.0 + (c - 2.0) * y * (1.0 - y));
}

static double rqf_slope(double y, double c)
{
    double den = 1.0 + (c - 2.0) * y * (1.0 - y);
    return (2.0 * y * (1.0 - y) + c * (1.0 - y) * (1.0 - y)) / (den * den);
}

double orc_rqf_inverse(double r, double c)
{
    double b = c - (c - 2.0) * r;
    return 2.0 * r / (b + sqrt(b * b + 4.0 * r * (1.0 - b)));
}

/* The fitted slopes c_k* for k = 1..7 (table tab:rambo_fit). */
double orc_rambo_ck(int32_t k)
{
    static const double ck[8] = {0.0, 2.0, 2.712001, 3.084521, 3.313073, 3.467512, 3.578833, 3.662872};
    return (k >= 1 && k <= 7) ? ck[k] : 0.0;
}

/* Mass of the (k + 1)-particle cluster Q_i: y = G_RQF^-1(r, c_k), u = y^(1/2k)
 * and M_i = mu_i + u (M_max - mu_i), with mu_i = sqrt(xmin) the sum of the
 * cluster's masses and M_max = sqrt(xmax) = M_{i-1} - m_{i-1} (its parent's
 * mass less its sibling's): for massless particles M_i = u_i M_{i-1}, the
 * construction of section 2.2.9; with masses, the massless chain of
 * K_i = M_i - mu_i.  Jacobian dM_i^2/dr = 2 M_i (M_max - mu_i) du/dr with
 * du/dr = u / (2 k y g_RQF(y, c_k)); with the decays' two-body factors the
 * product is the FastRambo mass measure (massive: with its reweighting). */
static double map_rambo(double r, int32_t k, double xmin, double xmax, double* jac)
{
    double c = orc_rambo_ck(k);
    double y = orc_rqf_inverse(r, c);
    double u = pow(y, 0.5 / k);
    double lo = sqrt(xmin), hi = sqrt(xmax);
    double m = lo + u * (hi - lo);
    *jac = 2.0 * m * (hi - lo) * u / (2.0 * k * y * rqf_slope(y, c));
    return m * m;
}

static double unmap_rambo(double x, int32_t k, double xmin, double xmax)
{
    double lo = sqrt(xmin), hi = sqrt(xmax);
    double u = (sqrt(x) - lo) / (hi - lo);
    return orc_rqf(pow(u, 2.0 * k), orc_rambo_ck(k));
}

/* Invariant of a propagator with mass m and width w: Breit-Wigner for w > 0,
 * otherwise G_nu; a massless structure gets the auxiliary m^2 = -a. */
static double map_invariant(double r, double m, double w, double nu, double reg_a,
                            double xmin, double xmax, double* jac)
{
    if (w > 0.0)
        return orc_map_bw(r, m, w, xmin, xmax, jac);
    double m2 = (m == 0.0) ? -reg_a : m * m;
    return orc_map_nu(r, m2, nu, xmin, xmax, jac);
}

/* Pure boost of k from the rest frame of P (mass m) to the frame in which P
 * has the given momentum. */
void orc_boost(const double P[4], double m, const double k[4], double out[4])
{
    double pk = P[1] * k[1] + P[2] * k[2] + P[3] * k[3];
    double e = (P[0] * k[0] + pk) / m;
    double c = (pk / (P[0] + m) + k[0]) / m;
    out[0] = e;
    out[1] = k[1] + c * P[1];
    out[2] = k[2] + c * P[2];
    out[3] = k[3] + c * P[3];
}

/* Rotation R(phi, theta) = R_z(phi) R_y(theta) (section 2.2.6) applied to v,
 * with the angles given by their cosines and sines. */
static void rotate(double cphi, double sphi, double cth, double sth, const double v[3], double out[3])
{
    double x = v[0] * cth + v[2] * sth;
    double y = v[1];
    double z = -v[0] * sth + v[2] * cth;
    out[0] = x * cphi - y * sphi;
    out[1] = x * sphi + y * cphi;
    out[2] = z;
}

/* Two-particle phase space in (phi, theta) (section 2.2.3, eq. ps2_phi_theta):
 * P of mass^2 m0sq decays into masses m1, m2; angles sampled uniformly in the
 * rest frame of P with fixed axes, then boosted back.  Returns the Jacobian
 * sqrt(lambda)/(8 m0^2) * 2pi * 2. */
double orc_two_body_decay(const double P[4], double m0sq, double m1, double m2,
                          double r_phi, double r_theta, double p1[4], double p2[4])
{
    double m0 = sqrt(m0sq);
    double m1s = m1 * m1, m2s = m2 * m2;
    double lam = orc_kallen(m0sq, m1s, m2s);
    double e1 = (m0sq + (m1s - m2s)) / (2.0 * m0);
    double e2 = (m0sq - (m1s - m2s)) / (2.0 * m0);
    double q = sqrt(lam) / (2.0 * m0);
    double phi = 2.0 * ORC_PI * r_phi;
    double cth = 2.0 * r_theta - 1.0;
    double sth = sqrt((1.0 - cth) * (1.0 + cth));
    double k1[4] = {e1, q * sth * cos(phi), q * sth * sin(phi), q * cth};
    double k2[4] = {e2, -k1[1], -k1[2], -k1[3]};
    orc_boost(P, m0, k1, p1);
    orc_boost(P, m0, k2, p2);
    return sqrt(lam) / (8.0 * m0sq) * (2.0 * ORC_PI) * 2.0;
}

/* Three-body decay P -> p1 + p2 + p3 (section 2.2.6): in the rest frame of P
 * (mass^2 m0sq) the energies E1 in [m1, E1max] and E2 in [E2min, E2max](E1)
 * linearly in r_e1, r_e2; the direction of p1 from (phi, cos theta) =
 * (2 pi r_phi, 2 r_theta - 1); p2 at the angle alpha to p1 that momentum
 * conservation fixes, turned by beta = 2 pi r_beta about p1; p3 = P - p1 -
 * p2; all boosted to the frame of P.  Returns the measure factor
 * (1/8) dE1 dE2 dphi dbeta dcos(theta) = pi^2 (E1max - m1)(E2max - E2min),
 * or 0 when the E2 range is empty; both widths are formed without
 * subtracting the range ends. */
double orc_three_body_decay(const double P[4], double m0sq, double m1, double m2, double m3, const double r[5],
                            double p1[4], double p2[4], double p3[4])
{
    const double m0 = sqrt(m0sq);
    /* E1max - m1 = ((m0 - m1)^2 - (m2 + m3)^2) / (2 m0), factored so that it
     * does not cancel near threshold */
    const double w1 = (m0 - m1 - (m2 + m3)) * (m0 - m1 + (m2 + m3)) / (2.0 * m0);
    const double e1 = m1 + w1 * r[0];
    const double q1 = sqrt(fmax(0.0, e1 * e1 - m1 * m1));
    /* the invariant mass^2 of p2 + p3, and the E2 range from its two-body
     * decay seen from the rest frame of P */
    const double dl = 2.0 * m0 * (0.5 * m0 - e1) + m1 * m1;
    const double d23 = m2 * m2 - m3 * m3;
    const double root = sqrt(fmax(0.0, q1 * q1 * ((dl + d23) * (dl + d23) - 4.0 * m2 * m2 * dl)));
    /* E2max - E2min = root / dl exactly: the width without the difference */
    const double e2min = ((m0 - e1) * (dl + d23) - root) / (2.0 * dl);
    const double w2 = root / dl;
    const double e2 = e2min + w2 * r[1];
    const double q2 = sqrt(fmax(0.0, e2 * e2 - m2 * m2));
    double ca = (2.0 * m0 * (0.5 * m0 - e1 - e2) + m1 * m1 + m2 * m2 + 2.0 * e1 * e2 - m3 * m3) / (2.0 * q1 * q2);
    if (!(ca >= -1.0)) ca = -1.0; /* rounding at the ends of the range (and 0/0) */
    if (ca > 1.0) ca = 1.0;
    const double sa = sqrt((1.0 - ca) * (1.0 + ca));
    const double phi = 2.0 * ORC_PI * r[2];
    const double ct = 2.0 * r[3] - 1.0;
    const double st = sqrt((1.0 - ct) * (1.0 + ct));
    const double beta = 2.0 * ORC_PI * r[4];
    const double cp = cos(phi), sp = sin(phi), cb = cos(beta), sb = sin(beta);
    /* R(phi, theta) = R_z(phi) R_y(theta) applied to a unit vector v */
    double v[3] = {cb * sa, sb * sa, ca};
    double w[3] = {ct * v[0] + st * v[2], v[1], -st * v[0] + ct * v[2]};
    double u2[3] = {cp * w[0] - sp * w[1], sp * w[0] + cp * w[1], w[2]};
    double u1[3] = {cp * st, sp * st, ct};
    double k1[4] = {e1, q1 * u1[0], q1 * u1[1], q1 * u1[2]};
    double k2[4] = {e2, q2 * u2[0], q2 * u2[1], q2 * u2[2]};
    double k3[4] = {m0 - e1 - e2, -k1[1] - k2[1], -k1[2] - k2[2], -k1[3] - k2[3]};
    orc_boost(P, m0, k1, p1);
    orc_boost(P, m0, k2, p2);
    orc_boost(P, m0, k3, p3);
    const double jac = ORC_PI * ORC_PI * w1 * w2;
    return jac > 0.0 ? jac : 0.0;
}

/* -t range of a 2->2 block (the t_inv_min_max operation): eq. t_invariant_theta
 * at cos(theta) = +1 and -1, for invariants m0^2 = (p_A + p_B)^2, ma^2 = p_A^2,
 * mb^2 = p_B^2 and outgoing masses m1, m2.  The root of smaller magnitude
 * (cos(theta) = +1), whose two terms cancel, is taken from the product of the
 * roots,
 *   t+ t- = (m1^2 - ma^2)(m2^2 - mb^2)
 *         + (ma^2 - mb^2 - m1^2 + m2^2)(ma^2 m2^2 - m1^2 mb^2) / m0^2,
 * which is exact algebra on the same two roots; it keeps |t|_min accurate
 * when it is far below the rounding noise of the other root (it is exactly 0
 * for massless external legs). */
void orc_t_range(double m0sq, double ma2, double mb2, double m1, double m2,
                 double* abst_min, double* abst_max)
{
    double m1s = m1 * m1, m2s = m2 * m2;
    double C = (m0sq + (m1s - m2s)) * (m0sq + (ma2 - mb2));
    double R = sqrt(orc_kallen(m0sq, m1s, m2s) * orc_kallen(m0sq, ma2, mb2));
    double prod = (m1s - ma2) * (m2s - mb2) + (ma2 - mb2 - m1s + m2s) * (ma2 * m2s - m1s * mb2) / m0sq;
    /* t at cos(theta) = -1 is the root of larger magnitude: evaluate it
     * directly, the other one from the product */
    double t_minus = m1s + ma2 - (C + R) / (2.0 * m0sq);
    double t_plus = (t_minus != 0.0) ? prod / t_minus : 0.0;
    *abst_min = fmax(0.0, -t_plus);
    *abst_max = -t_minus;
}

/* Two-particle phase space in (phi, t) (section 2.2.4, eqs. t_invariant_theta,
 * 2_to_2_mapping, ps2_phi_t).  p_A, p_B fix the frame; their invariants
 * m0sq = (p_A + p_B)^2, ma2 = p_A^2, mb2 = p_B^2 are the values already
 * sampled upstream (s-hat or a time-like invariant, and the |t| of earlier
 * blocks), which the momenta satisfy up to rounding.
 * |t| = G_nu(r_t; 0, |t|_min, |t|_max) with the auxiliary mass of a massless
 * t-propagator; theta is measured from the direction of p_A in the rest
 * frame of P = p_A + p_B, phi around it.
 * Returns J_t * 2pi / (4 sqrt(lambda(m0^2, ma^2, mb^2))); *abst receives |t|. */
double orc_two_to_two(const double pA[4], const double pB[4], double m0sq, double ma2, double mb2,
                      double m1, double m2, double r_phi, double r_t, double nu, double reg_a,
                      double p1[4], double p2[4], double* abst_out)
{
    double P[4] = {pA[0] + pB[0], pA[1] + pB[1], pA[2] + pB[2], pA[3] + pB[3]};
    double m0 = sqrt(m0sq);
    double m1s = m1 * m1, m2s = m2 * m2;
    double lam12 = orc_kallen(m0sq, m1s, m2s), lamab = orc_kallen(m0sq, ma2, mb2);
    double C = (m0sq + (m1s - m2s)) * (m0sq + (ma2 - mb2));
    double R = sqrt(lam12 * lamab);
    double tmin_abs, tmax_abs;
    orc_t_range(m0sq, ma2, mb2, m1, m2, &tmin_abs, &tmax_abs);
    double jt;
    double abst = orc_map_nu(r_t, -reg_a, nu, tmin_abs, tmax_abs, &jt);
    /* invert eq. t_invariant_theta for cos(theta) */
    double cth = (C - 2.0 * m0sq * (m1s + ma2 + abst)) / R;
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    double sth = sqrt((1.0 - cth) * (1.0 + cth));
    double phi = 2.0 * ORC_PI * r_phi;
    double q = sqrt(lam12) / (2.0 * m0);
    double e1 = (m0sq + (m1s - m2s)) / (2.0 * m0);
    double e2 = (m0sq - (m1s - m2s)) / (2.0 * m0);
    double v1[3] = {q * sth * cos(phi), q * sth * sin(phi), q * cth};
    /* direction of p_A in the rest frame of P */
    double Pbar[4] = {P[0], -P[1], -P[2], -P[3]};
    double pAr[4];
    orc_boost(Pbar, m0, pA, pAr);
    double len = sqrt(pAr[1] * pAr[1] + pAr[2] * pAr[2] + pAr[3] * pAr[3]);
    double nx = pAr[1] / len, ny = pAr[2] / len, nz = pAr[3] / len;
    double st = sqrt(nx * nx + ny * ny);
    double cp = 1.0, sp = 0.0;
    if (st > 0.0) {
        cp = nx / st;
        sp = ny / st;
    }
    double w1[3];
    rotate(cp, sp, nz, st, v1, w1);
    double k1[4] = {e1, w1[0], w1[1], w1[2]};
    double k2[4] = {e2, -w1[0], -w1[1], -w1[2]};
    orc_boost(P, m0, k1, p1);
    orc_boost(P, m0, k2, p2);
    if (abst_out) *abst_out = abst;
    return jt * (2.0 * ORC_PI) / (4.0 * sqrt(lamab));
}

double orc_unmap_nu(double x, double m2, double nu, double xmin, double xmax);

/* Inverse of rotate (R(phi, theta)^-1 = R_y(-theta) R_z(-phi)). */
static void unrotate(double cphi, double sphi, double cth, double sth, const double v[3], double out[3])
{
    double x = v[0] * cphi + v[1] * sphi;
    double y = -v[0] * sphi + v[1] * cphi;
    out[0] = x * cth - v[2] * sth;
    out[1] = y;
    out[2] = x * sth + v[2] * cth;
}

/* The (s~, t) double-invariant block (section 2.2.5, eqs. byckling,
 * t_invariant_theta_23, s_to_phi): as the (phi, t) block, P = p_A + p_B of
 * mass^2 m0sq goes to p1 (mass m1, the leg next to A) and p2 (mass m2) with
 * |t| = -(p_A - p1)^2 from G_nu, but the azimuth of p1 about p_A in the rest
 * frame of P is fixed by the time-like invariant s~ = (p1 + rec)^2 of p1
 * and the recoil momentum rec (the leg the previous block peeled on this
 * side), measured from the plane of p_A and rec.  In that frame s~ = A - B
 * cos(phi) with A = m1^2 + rec^2 + 2 (E1 E_rec - |p1| cos(theta) rec_z),
 * B = 2 |p1| sin(theta) |rec_perp|, so s~ is linear in r between A - B and
 * A + B.  s~ fixes cos(phi) only (reading): the half of [0, 1) that r_s
 * falls in gives the sign of sin(phi), and r_s rescaled to the half gives s~.
 * Measure: d|t| dphi / (4 sqrt(lambda_ab)) as in the (phi, t) block, with
 * dphi = ds~ / (B |sin phi|) per branch -- on each branch the paper's density
 * 1 / (8 sqrt(-Delta_4)) in ds~ d|t| (here sqrt(-Delta_4) = sqrt(lambda_ab) B
 * |sin phi| / 2), so the two branches together carry twice it.  Jacobian
 * dr_s d r_t -> phase space: J_|t| / (sqrt(lambda_ab) |sin phi|).  *stil_out
 * (optional) receives s~. */
double orc_two_to_two_st(const double pA[4], const double pB[4], const double rec[4], double m0sq, double ma2,
                         double mb2, double m1, double m2, double r_s, double r_t, double nu, double reg_a,
                         double p1[4], double p2[4], double* abst_out, double* stil_out)
{
    double P[4] = {pA[0] + pB[0], pA[1] + pB[1], pA[2] + pB[2], pA[3] + pB[3]};
    double m0 = sqrt(m0sq);
    double m1s = m1 * m1, m2s = m2 * m2;
    double lam12 = orc_kallen(m0sq, m1s, m2s), lamab = orc_kallen(m0sq, ma2, mb2);
    double C = (m0sq + (m1s - m2s)) * (m0sq + (ma2 - mb2));
    double R = sqrt(lam12 * lamab);
    double tmin_abs, tmax_abs;
    orc_t_range(m0sq, ma2, mb2, m1, m2, &tmin_abs, &tmax_abs);
    double jt;
    double abst = orc_map_nu(r_t, -reg_a, nu, tmin_abs, tmax_abs, &jt);
    double cth = (C - 2.0 * m0sq * (m1s + ma2 + abst)) / R;
    if (cth > 1.0) cth = 1.0;
    if (cth < -1.0) cth = -1.0;
    double sth = sqrt((1.0 - cth) * (1.0 + cth));
    double q = sqrt(lam12) / (2.0 * m0);
    double e1 = (m0sq + (m1s - m2s)) / (2.0 * m0);
    double e2 = (m0sq - (m1s - m2s)) / (2.0 * m0);
    /* p_A along z in the rest frame of P */
    double Pbar[4] = {P[0], -P[1], -P[2], -P[3]};
    double pAr[4];
    orc_boost(Pbar, m0, pA, pAr);
    double len = sqrt(pAr[1] * pAr[1] + pAr[2] * pAr[2] + pAr[3] * pAr[3]);
    double nx = pAr[1] / len, ny = pAr[2] / len, nz = pAr[3] / len;
    double st = sqrt(nx * nx + ny * ny);
    double cp = 1.0, sp = 0.0;
    if (st > 0.0) {
        cp = nx / st;
        sp = ny / st;
    }
    /* the recoil in the same frame */
    double recr[4], rz[3];
    orc_boost(Pbar, m0, rec, recr);
    unrotate(cp, sp, nz, st, recr + 1, rz);
    double rperp = sqrt(rz[0] * rz[0] + rz[1] * rz[1]);
    double mrec2 = rec[0] * rec[0] - rec[1] * rec[1] - rec[2] * rec[2] - rec[3] * rec[3];
    double A = m1s + mrec2 + 2.0 * (e1 * recr[0] - q * cth * rz[2]);
    double B = 2.0 * q * sth * rperp;
    double sgn = 1.0, u = 2.0 * r_s;
    if (r_s >= 0.5) {
        sgn = -1.0;
        u = 2.0 * r_s - 1.0;
    }
    double stil = (A - B) + 2.0 * B * u;
    /* eq. s_to_phi inverted: cos(phi) = (A - s~) / B, which for s~ linear in
     * u is exactly 1 - 2 u (formed so, without A cancelling against s~) */
    double cphi = 1.0 - 2.0 * u;
    double sphi = sgn * 2.0 * sqrt(u * (1.0 - u));
    /* azimuth of p1 = that of the recoil plus phi */
    double ux = rz[0] / rperp, uy = rz[1] / rperp;
    double c1 = ux * cphi - uy * sphi, s1 = uy * cphi + ux * sphi;
    double v1[3] = {q * sth * c1, q * sth * s1, q * cth};
    double w1[3];
    rotate(cp, sp, nz, st, v1, w1);
    double k1[4] = {e1, w1[0], w1[1], w1[2]};
    double k2[4] = {e2, -w1[0], -w1[1], -w1[2]};
    orc_boost(P, m0, k1, p1);
    orc_boost(P, m0, k2, p2);
    if (abst_out) *abst_out = abst;
    if (stil_out) *stil_out = stil;
    return jt / (sqrt(lamab) * fabs(sphi));
}

/* Inverse of orc_two_to_two_st: from p1 (and p_A, p_B, rec) the uniforms
 * (r_s, r_t). */
void orc_two_to_two_st_inverse(const double pA[4], const double pB[4], const double rec[4], double m0sq,
                               double ma2, double mb2, double m1, double m2, const double p1[4], double nu,
                               double reg_a, double* r_s, double* r_t)
{
    double P[4] = {pA[0] + pB[0], pA[1] + pB[1], pA[2] + pB[2], pA[3] + pB[3]};
    double m0 = sqrt(m0sq);
    double m1s = m1 * m1, m2s = m2 * m2;
    double lam12 = orc_kallen(m0sq, m1s, m2s);
    double d[4] = {pA[0] - p1[0], pA[1] - p1[1], pA[2] - p1[2], pA[3] - p1[3]};
    double abst = -(d[0] * d[0] - d[1] * d[1] - d[2] * d[2] - d[3] * d[3]);
    double tmin_abs, tmax_abs;
    orc_t_range(m0sq, ma2, mb2, m1, m2, &tmin_abs, &tmax_abs);
    *r_t = orc_unmap_nu(abst, -reg_a, nu, tmin_abs, tmax_abs);
    double q = sqrt(lam12) / (2.0 * m0);
    double e1 = (m0sq + (m1s - m2s)) / (2.0 * m0);
    double Pbar[4] = {P[0], -P[1], -P[2], -P[3]};
    double pAr[4], recr[4], k1[4];
    orc_boost(Pbar, m0, pA, pAr);
    orc_boost(Pbar, m0, rec, recr);
    orc_boost(Pbar, m0, p1, k1);
    double len = sqrt(pAr[1] * pAr[1] + pAr[2] * pAr[2] + pAr[3] * pAr[3]);
    double nx = pAr[1] / len, ny = pAr[2] / len, nz = pAr[3] / len;
    double st = sqrt(nx * nx + ny * ny);
    double cp = 1.0, sp = 0.0;
    if (st > 0.0) {
        cp = nx / st;
        sp = ny / st;
    }
    double rz[3], kz[3];
    unrotate(cp, sp, nz, st, recr + 1, rz);
    unrotate(cp, sp, nz, st, k1 + 1, kz);
    double rperp = sqrt(rz[0] * rz[0] + rz[1] * rz[1]);
    double kperp = sqrt(kz[0] * kz[0] + kz[1] * kz[1]);
    /* u = (s~ - (A - B)) / (2 B) = (1 - cos(phi)) / 2 with phi the angle
     * between the transverse parts of the recoil and p1 (formed from them,
     * without the cancellation of s~ against A); the branch from the
     * orientation of p1 about the plane of p_A and the recoil */
    double cphi = (rz[0] * kz[0] + rz[1] * kz[1]) / (rperp * kperp);
    if (cphi > 1.0) cphi = 1.0;
    if (cphi < -1.0) cphi = -1.0;
    double cross = rz[0] * kz[1] - rz[1] * kz[0];
    double u = 0.5 * (1.0 - cphi);
    *r_s = cross >= 0.0 ? 0.5 * u : 0.5 * (u + 1.0);
    (void)q;
    (void)e1;
}

/* PDF convolution (section 2.2.2, eqs. pdf_conv, pdf_sampling): x1 = tau^r,
 * x2 = tau^(1-r), Jacobian -log(tau)/s_lab (the r_to_x1x2 operation). */
double orc_r_to_x1x2(double r, double shat, double s_lab, double* x1, double* x2)
{
    double tau = shat / s_lab;
    *x1 = pow(tau, r);
    *x2 = pow(tau, 1.0 - r);
    return -log(tau) / s_lab;
}

/* VEGAS map of one uniform y through a grid with nb bins (edges e_0..e_nb):
 * bin i = floor(y nb), linear inside the bin, Jacobian nb (e_{i+1} - e_i). */
double orc_vegas_map(double y, const double* edges, int32_t nb, double* jac)
{
    double t = y * nb;
    int32_t i = (int32_t)floor(t);
    if (i > nb - 1) i = nb - 1;
    if (i < 0) i = 0;
    double wdt = edges[i + 1] - edges[i];
    *jac = nb * wdt;
    return edges[i] + wdt * (t - i);
}

/* ------------------------------------------------------------------------ */
/* s-channel integration order bounds (section 2.2.7)                        */
/* ------------------------------------------------------------------------ */

static double node_m_min(const orc_channel* ch, int32_t j, const int32_t* sampled, const double* s)
{
    if (ch->kind[j] == ORC_LEAF) return ch->mass[j];
    if (sampled[j]) return sqrt(s[j]);
    double sum = 0.0;
    for (int32_t c = 0; c < ch->child_count[j]; ++c)
        sum += node_m_min(ch, ch->children[ch->child_start[j] + c], sampled, s);
    return sum;
}

/* Walk from node i towards the root until a sampled node r is met and
 * subtract the minimal masses of everything that branches off the path
 * (children of r included, children of i excluded). */
static double node_m_max(const orc_channel* ch, int32_t i, const int32_t* sampled, const double* s)
{
    double sub = 0.0;
    int32_t v = i;
    while (!sampled[v]) {
        int32_t par = ch->parent[v];
        for (int32_t c = 0; c < ch->child_count[par]; ++c) {
            int32_t sib = ch->children[ch->child_start[par] + c];
            if (sib != v) sub += node_m_min(ch, sib, sampled, s);
        }
        v = par;
    }
    return sqrt(s[v]) - sub;
}

/* ------------------------------------------------------------------------ */
/* One event                                                                 */
/* ------------------------------------------------------------------------ */

static double pdf_toy(const orc_process* pr, double x)
{
    return pow(x, pr->pdf_a) * pow(1.0 - x, pr->pdf_b + (ORC_MUTATE == 1 ? 1.0 : 0.0));
}

static double prop_q2(int32_t t_type, uint32_t set, const double pa[4], double mom[][4], int32_t n)
{
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t k = 0; k < n; ++k)
        if (set & (1u << k))
            for (int c = 0; c < 4; ++c) q[c] += mom[k][c];
    if (t_type)
        for (int c = 0; c < 4; ++c) q[c] = ORC_MUTATE == 3 ? pa[c] + q[c] : pa[c] - q[c];
    return mdot(q, q);
}

/* Integrand f (the toy integrand: PDFs, pT cut, 1 + cos^2, propagator factors) and
 * the local channel weight alpha_c(x) = P_c / sum_c' P_c' (eq.
 * multi-channel-mg, weights from propagator denominators) of final-state
 * momenta pf[n] and incoming p_a. */
static double integrand(const orc_process* pr, int32_t chan, double pf[][4], const double pa[4],
                        double x1, double x2, double* alpha_out)
{
    const int32_t n = pr->n_final;
    double f = 1.0, alpha;
    if (pr->pdf) f *= pdf_toy(pr, x1) * pdf_toy(pr, x2);
    if (pr->pt_min > 0.0)
        for (int32_t i = 0; i < n; ++i)
            if (!(pf[i][1] * pf[i][1] + pf[i][2] * pf[i][2] > pr->pt_min * pr->pt_min)) f = 0.0;
    if (pr->ang >= 0) {
        const double* p = pf[pr->ang];
        double c = p[3] / sqrt(p[1] * p[1] + p[2] * p[2] + p[3] * p[3]);
        f *= 1.0 + c * c;
    }
    for (int32_t u = 0; u < pr->n_prop; ++u) {
        double q2 = prop_q2(pr->prop_t[u], pr->prop_set[u], pa, pf, n);
        if (pr->prop_bw[u]) {
            double m2 = pr->prop_m[u] * pr->prop_m[u], mw = pr->prop_m[u] * pr->prop_w[u];
            if (ORC_MUTATE == 4) mw = pr->prop_w[u];
            f *= 1.0 / ((q2 - m2) * (q2 - m2) + mw * mw);
        } else {
            f *= 1.0 / (fabs(q2) + (ORC_MUTATE == 2 ? pr->prop_mu[u] : pr->prop_mu[u] * pr->prop_mu[u]));
        }
    }
    if (pr->n_chan <= 1) {
        alpha = 1.0;
    } else if (pr->ch_prior && pr->ch_prior[chan]) {
        /* a channel without a diagram has no propagator denominators to
         * weigh: it takes the constant share 1 / n_chan */
        alpha = 1.0 / pr->n_chan;
    } else {
        double den = 0.0, mine = 0.0, share = 1.0;
        for (int32_t c = 0; c < pr->n_chan; ++c) {
            if (pr->ch_prior && pr->ch_prior[c]) {
                share -= 1.0 / pr->n_chan;
                continue;
            }
            double P = 1.0;
            for (int32_t u = pr->ch_start[c]; u < pr->ch_start[c + 1]; ++u) {
                double q2 = prop_q2(pr->chp_t[u], pr->chp_set[u], pa, pf, n);
                double m = pr->chp_m[u];
                if (m > 0.0) {
                    double mw = m * pr->chp_w[u];
                    P *= 1.0 / ((q2 - m * m) * (q2 - m * m) + mw * mw);
                } else {
                    double d = fabs(q2) + pr->alpha_mu * pr->alpha_mu;
                    P *= 1.0 / (d * d);
                }
            }
            den += P;
            if (c == chan) mine = P;
        }
        /* the diagram channels share what the others leave, in proportion
         * to their propagator products */
        alpha = share * (mine / den);
    }
    *alpha_out = alpha;
    return f;
}

typedef struct {
    double p[ORC_MAX_FINAL + 2][4]; /* lab frame: a, b, 1..n */
    double x1, x2, jac, w, alpha, f;
    double inv[ORC_MAX_NODES];      /* sampled invariants per node (0 if none) */
    double tabs[ORC_MAX_FINAL];     /* |t| sampled by each 2->2 block, in order */
} orc_event;

/* The whole per-event chain for channel `chan` of process `pr`, given the
 * uniforms y[d] (before VEGAS) and the channel's VEGAS grid (NULL: none). */
static void event_tail(const orc_process* pr, int32_t chan, double pf[][4], const double pa[4], const double pb[4],
                       double x1, double x2, const double* factors, int32_t nf, orc_event* ev);
static void event_chili(const orc_process* pr, int32_t chan, const double* r, double jv, orc_event* ev);

static void event(const orc_process* pr, const orc_channel* ch, int32_t chan,
                  const double* y, int32_t dims, const double* grid, int32_t nb, orc_event* ev)
{
    const int32_t n = pr->n_final;
    double r[ORC_MAX_DIMS];
    double jv = 1.0;
    for (int32_t k = 0; k < dims; ++k) {
        if (grid) {
            double jk;
            r[k] = orc_vegas_map(y[k], grid + (size_t)k * (nb + 1), nb, &jk);
            jv *= jk;
        } else {
            r[k] = y[k];
        }
    }
    if (ch->chili) {
        event_chili(pr, chan, r, jv, ev);
        return;
    }

    double s[ORC_MAX_NODES];
    int32_t sampled[ORC_MAX_NODES];
    double mom[ORC_MAX_NODES][4];
    for (int32_t j = 0; j < ch->n_nodes; ++j) {
        s[j] = 0.0;
        sampled[j] = 0;
        ev->inv[j] = 0.0;
    }
    double factors[4 * ORC_MAX_FINAL + 8];
    int32_t nf = 0;
    factors[nf++] = pow(2.0 * ORC_PI, 4.0 - 3.0 * n); /* (2pi)^(4-3n), section 2.2 */

    int32_t k = 0; /* dimension cursor */
    const int32_t root = ch->root;

    /* (1) s-hat: power-law map (or Breit-Wigner for a resonant pure-s root)
     *     on [shat_min, s_lab]; fixed for lepton beams. */
    double shat;
    if (pr->hadronic) {
        double m = 0.0, w = 0.0, nu = pr->nu;
        if (ch->kind[root] == ORC_CLUSTER) {
            m = ch->mass[root];
            w = ch->width[root];
            nu = ch->nu[root];
        }
        double lo = pr->shat_min;
        double msum = 0.0;
        for (int32_t i = 0; i < n; ++i) msum += pr->mass[i];
        if (msum * msum > lo) lo = msum * msum;
        double js;
        shat = map_invariant(r[k++], m, w, nu, pr->reg_a, lo, pr->s_lab, &js);
        factors[nf++] = js;
    } else {
        shat = pr->s_lab;
    }
    s[root] = shat;
    sampled[root] = 1;
    ev->inv[root] = shat;

    /* (2) time-like invariants of the decay clusters in the channel's order,
     *     bounds from the minimal/maximal mass recursion (section 2.2.7). */
    for (int32_t q = 0; q < ch->n_sorder; ++q) {
        int32_t i = ch->s_order[q];
        double mmin = 0.0;
        for (int32_t c = 0; c < ch->child_count[i]; ++c)
            mmin += node_m_min(ch, ch->children[ch->child_start[i] + c], sampled, s);
        double mmax = node_m_max(ch, i, sampled, s);
        double ji;
        if (ch->rambo && ch->rambo[i] > 0)
            s[i] = map_rambo(r[k++], ch->rambo[i], mmin * mmin, mmax * mmax, &ji);
        else
            s[i] = map_invariant(r[k++], ch->mass[i], ch->width[i], ch->nu[i], pr->reg_a,
                                 mmin * mmin, mmax * mmax, &ji);
        sampled[i] = 1;
        ev->inv[i] = s[i];
        factors[nf++] = ji;
    }

    /* (3) t-channel: generation order sigma from the A/B choices, then the
     *     kappa-1 time-like invariants s_1..s_{kappa-1} (section 2.2.8). */
    int32_t kappa = 0;
    int32_t sigma[ORC_MAX_FINAL + 1];
    int32_t from_a[ORC_MAX_FINAL + 1];
    double st[ORC_MAX_FINAL + 1]; /* s_0 .. s_{kappa-1} */
    if (ch->kind[root] == ORC_TNODE) {
        kappa = ch->child_count[root] - 1;
        const int32_t* legs = ch->children + ch->child_start[root];
        int32_t lo = 0, hi = kappa;
        for (int32_t i = 1; i < kappa; ++i) {
            if (ch->t_order[i - 1] == 'A') {
                sigma[i] = legs[lo++];
                from_a[i] = 1;
            } else {
                sigma[i] = legs[hi--];
                from_a[i] = 0;
            }
        }
        sigma[kappa] = legs[lo];
        sigma[kappa + 1] = legs[hi];
        st[0] = shat;
        for (int32_t i = 1; i < kappa; ++i) {
            double msum = 0.0;
            for (int32_t j = i + 1; j <= kappa + 1; ++j) msum += node_m_min(ch, sigma[j], sampled, s);
            double mi = node_m_min(ch, sigma[i], sampled, s);
            double smin = msum * msum;
            double dm = sqrt(st[i - 1]) - mi;
            double ji;
            st[i] = map_invariant(r[k++], 0.0, 0.0, pr->nu, pr->reg_a, smin, dm * dm, &ji);
            factors[nf++] = ji;
        }
    }

    /* (4) momentum fractions */
    double x1 = 1.0, x2 = 1.0;
    if (pr->hadronic) {
        double jx = orc_r_to_x1x2(r[k++], shat, pr->s_lab, &x1, &x2);
        factors[nf++] = jx;
    }

    /* (5) incoming momenta in the partonic centre-of-mass frame (com_p_in) */
    double rs = sqrt(shat);
    double pa[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs};
    double pb[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};

    /* (6) chain of 2->2 blocks with the corrected leg update: peeling the leg
     *     next to A replaces p_A by p_A - p1, next to B replaces p_B by p_B - p2. */
    if (ch->kind[root] == ORC_TNODE) {
        double pA[4], pB[4];
        memcpy(pA, pa, sizeof pA);
        memcpy(pB, pb, sizeof pB);
        double ma2 = 0.0, mb2 = 0.0; /* p_A^2, p_B^2: 0, then the t of the block that updated them */
        for (int32_t i = 1; i <= kappa; ++i) {
            double m1, m2;
            if (i == kappa) {
                m1 = node_m_min(ch, sigma[kappa], sampled, s);
                m2 = node_m_min(ch, sigma[kappa + 1], sampled, s);
            } else if (from_a[i]) {
                m1 = node_m_min(ch, sigma[i], sampled, s);
                m2 = sqrt(st[i]);
            } else {
                m1 = sqrt(st[i]);
                m2 = node_m_min(ch, sigma[i], sampled, s);
            }
            double r_phi = r[k++], r_t = r[k++];
            double p1[4], p2[4];
            /* with st, a block after the first replaces phi by s~ = (p1 +
             * the leg the previous block peeled)^2 */
            double jb = (ch->st && i >= 2)
                            ? orc_two_to_two_st(pA, pB, mom[sigma[i - 1]], st[i - 1], ma2, mb2, m1, m2, r_phi, r_t,
                                                pr->nu, pr->reg_a, p1, p2, &ev->tabs[i - 1], NULL)
                            : orc_two_to_two(pA, pB, st[i - 1], ma2, mb2, m1, m2, r_phi, r_t, pr->nu,
                                             pr->reg_a, p1, p2, &ev->tabs[i - 1]);
            factors[nf++] = jb;
            if (i == kappa) {
                memcpy(mom[sigma[kappa]], p1, sizeof p1);
                memcpy(mom[sigma[kappa + 1]], p2, sizeof p2);
            } else if (from_a[i]) {
                memcpy(mom[sigma[i]], p1, sizeof p1);
                for (int c = 0; c < 4; ++c) pA[c] -= p1[c];
                ma2 = -ev->tabs[i - 1];
            } else {
                memcpy(mom[sigma[i]], p2, sizeof p2);
                for (int c = 0; c < 4; ++c) pB[c] -= p2[c];
                mb2 = -ev->tabs[i - 1];
            }
        }
    } else {
        mom[root][0] = rs;
        mom[root][1] = mom[root][2] = mom[root][3] = 0.0;
    }

    /* (7) (phi, theta) decays of the clusters, parents before children */
    for (int32_t q = 0; q < ch->n_dec; ++q) {
        int32_t c = ch->dec_order[q];
        int32_t c0 = ch->children[ch->child_start[c]], c1 = ch->children[ch->child_start[c] + 1];
        double m1 = node_m_min(ch, c0, sampled, s), m2 = node_m_min(ch, c1, sampled, s);
        if (ch->child_count[c] == 3) {
            /* 1 -> 3 decay: dimensions (E1, E2, phi, theta, beta) */
            int32_t c2 = ch->children[ch->child_start[c] + 2];
            double m3 = node_m_min(ch, c2, sampled, s);
            double jd = orc_three_body_decay(mom[c], s[c], m1, m2, m3, r + k, mom[c0], mom[c1], mom[c2]);
            k += 5;
            factors[nf++] = jd;
            continue;
        }
        double r_phi = r[k++], r_theta = r[k++];
        double jd = orc_two_body_decay(mom[c], s[c], m1, m2, r_phi, r_theta, mom[c0], mom[c1]);
        factors[nf++] = jd;
    }
    factors[nf++] = 1.0; /* channel constant */
    factors[nf++] = jv;  /* VEGAS Jacobian */

    /* final-state momenta in the partonic frame, by particle label */
    double pf[ORC_MAX_FINAL][4];
    for (int32_t j = 0; j < ch->n_nodes; ++j)
        if (ch->kind[j] == ORC_LEAF) memcpy(pf[ch->particle[j]], mom[j], sizeof pf[0]);
    event_tail(pr, chan, pf, pa, pb, x1, x2, factors, nf, ev);
}

/* Steps (8)-(11) of an event whose final-state momenta pf are in the
 * partonic frame (incoming pa, pb): beam boost, reduce_product of the
 * Jacobian factors, cut_unphysical, integrand and channel weight. */
static void event_tail(const orc_process* pr, int32_t chan, double pf[][4], const double pa[4], const double pb[4],
                       double x1, double x2, const double* factors, int32_t nf, orc_event* ev)
{
    const int32_t n = pr->n_final;
#ifdef ORC_LIBM_NUDGE
    /* perturbation builds: move every component by one ulp, alternating in
     * direction, so that quantities recomputed from the momenta see a
     * rounding-size change of the momenta themselves */
    for (int32_t i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c)
            if (pf[i][c] != 0.0)
                pf[i][c] = nextafter(pf[i][c], ((i + c + (ORC_LIBM_NUDGE > 0)) & 1) ? INFINITY : -INFINITY);
#endif

    /* (8) boost_beam: longitudinal boost to the lab frame */
    double g = 1.0, gb = 0.0;
    if (pr->hadronic) {
        double sq = sqrt(x1 * x2);
        g = (x1 + x2) / (2.0 * sq);
        gb = (x1 - x2) / (2.0 * sq);
    }
    double (*out)[4] = ev->p;
    const double* src[ORC_MAX_FINAL + 2];
    src[0] = pa;
    src[1] = pb;
    for (int32_t i = 0; i < n; ++i) src[i + 2] = pf[i];
    for (int32_t i = 0; i < n + 2; ++i) {
        out[i][0] = g * src[i][0] + gb * src[i][3];
        out[i][1] = src[i][1];
        out[i][2] = src[i][2];
        out[i][3] = gb * src[i][0] + g * src[i][3];
    }

    /* (9) reduce_product of all Jacobian factors, left to right */
    double jac = 1.0;
    for (int32_t i = 0; i < nf; ++i) jac *= factors[i];

    /* (10) cut_unphysical: non-finite values, momentum fractions outside
     *      (0, 1], negative energies or a non-positive Jacobian -> weight 0 */
    int ok = isfinite(jac) && jac > 0.0;
    for (int32_t i = 0; i < n + 2 && ok; ++i)
        for (int c = 0; c < 4; ++c)
            if (!isfinite(out[i][c])) ok = 0;
    for (int32_t i = 0; i < n + 2 && ok; ++i)
        if (out[i][0] < 0.0) ok = 0;
    if (pr->hadronic && ok)
        if (!(isfinite(x1) && isfinite(x2) && x1 > 0.0 && x1 <= 1.0 && x2 > 0.0 && x2 <= 1.0)) ok = 0;
    if (!ok) jac = 0.0;

    /* (11) integrand f and local channel weight alpha_c(x) (SDE multichannel,
     *      eq. multi-channel-mg) from invariants of the partonic-frame momenta */
    double f = 0.0, alpha = 0.0;
    if (ok) f = integrand(pr, chan, pf, pa, x1, x2, &alpha);
    ev->x1 = x1;
    ev->x2 = x2;
    ev->jac = jac;
    ev->f = f;
    ev->alpha = alpha;
    ev->w = alpha * f * jac;
}

/* ------------------------------------------------------------------------ */
/* Chili (section 2.4)                                                       */
/* ------------------------------------------------------------------------ */

/* One Chili event: particles 1..n-1 from (p_T, y, phi) in the lab frame --
 * p_T^2 by the 1/p_T^2 map between the process's p_T cut and sqrt(s_lab)/2
 * (eq. chili_pt_withcut), or without a cut the regulated map of eq.
 * chili_pt_nocut (lambda = m, 1 for massless); y uniform in +-y_max(m_T);
 * phi uniform, measured from the current recoil direction -- then the last
 * particle's transverse momentum by recoil and its rapidity uniform in the
 * range the beam energy leaves, and x_1,2 = E^+- / sqrt(s_lab).  Measure:
 * integrating dx1 dx2 prod d^3p / 2E against the momentum delta leaves
 * (2 pi)^(4-3n) / s_lab dy_n prod_(i<n) dp_T^2 dy dphi / 4; each factor is
 * the exact derivative of its map.  Dimensions per particle (p_T, y, phi),
 * then y_n. */
static void event_chili(const orc_process* pr, int32_t chan, const double* r, double jv, orc_event* ev)
{
    const int32_t n = pr->n_final;
    const double sq = sqrt(pr->s_lab), ptmax = 0.5 * sq;
    double pl[ORC_MAX_FINAL][4];
    double factors[4 * ORC_MAX_FINAL + 8];
    int32_t nf = 0;
    factors[nf++] = pow(2.0 * ORC_PI, 4.0 - 3.0 * n) / pr->s_lab;
    double sx = 0.0, sy = 0.0, ep = 0.0, em = 0.0;
    int32_t k = 0;
    int ok = 1;
    for (int32_t i = 0; i < n - 1; ++i) {
        const double m = pr->mass[i];
        double pt2, jpt2;
        const double rp = r[k++];
        if (pr->pt_min > 0.0) {
            const double a = 1.0 / (ptmax * ptmax), b = 1.0 / (pr->pt_min * pr->pt_min);
            pt2 = 1.0 / (rp * a + (1.0 - rp) * b);
            jpt2 = (b - a) * pt2 * pt2;
        } else {
            const double lam = m > 0.0 ? m : 1.0;
            const double den = 2.0 * lam + ptmax * (1.0 - rp);
            const double pt = 2.0 * lam * ptmax * rp / den;
            pt2 = pt * pt;
            jpt2 = 2.0 * pt * 2.0 * lam * ptmax * (2.0 * lam + ptmax) / (den * den);
        }
        const double mt = sqrt(pt2 + m * m);
        const double z = sq / (2.0 * mt);
        if (!(z > 1.0)) ok = 0;
        const double ymax = ok ? log(z + sqrt(z * z - 1.0)) : 0.0;
        const double yv = ymax * (2.0 * r[k++] - 1.0);
        const double phi_rec = (i == 0) ? 0.0 : atan2(-sy, -sx);
        const double phi = 2.0 * ORC_PI * r[k++] + phi_rec;
        const double pt = sqrt(pt2);
        /* E +- p_z = m_T exp(+-y): the light-cone components without cancellation */
        const double lp = mt * exp(yv), lm = mt * exp(-yv);
        pl[i][0] = 0.5 * (lp + lm);
        pl[i][1] = pt * cos(phi);
        pl[i][2] = pt * sin(phi);
        pl[i][3] = 0.5 * (lp - lm);
        sx += pl[i][1];
        sy += pl[i][2];
        ep += lp;
        em += lm;
        factors[nf++] = jpt2 * (2.0 * ymax) * (2.0 * ORC_PI) / 4.0;
    }
    /* the last particle: recoil, rapidity within the beam energy */
    {
        const int32_t i = n - 1;
        const double m = pr->mass[i];
        const double px = -sx, py = -sy;
        const double mt = sqrt(px * px + py * py + m * m);
        const double ylo = -log((sq - em) / mt), yhi = log((sq - ep) / mt);
        if (!(sq > ep && sq > em && yhi > ylo)) ok = 0;
        const double yv = ok ? ylo + (yhi - ylo) * r[k++] : 0.0;
        const double lp = mt * exp(yv), lm = mt * exp(-yv);
        pl[i][0] = 0.5 * (lp + lm);
        pl[i][1] = px;
        pl[i][2] = py;
        pl[i][3] = 0.5 * (lp - lm);
        ep += lp;
        em += lm;
        factors[nf++] = ok ? (yhi - ylo) : 0.0;
    }
    factors[nf++] = 1.0; /* channel constant */
    factors[nf++] = jv;
    double x1 = ep / sq, x2 = em / sq;
    if (!ok) x1 = x2 = 0.5; /* any values: the zero factor cuts the event */
    /* the partonic frame: undo the beam boost of x1, x2 */
    const double sqx = sqrt(x1 * x2);
    const double g = (x1 + x2) / (2.0 * sqx), gb = (x1 - x2) / (2.0 * sqx);
    double pf[ORC_MAX_FINAL][4];
    for (int32_t i = 0; i < n; ++i) {
        pf[i][0] = g * pl[i][0] - gb * pl[i][3];
        pf[i][1] = pl[i][1];
        pf[i][2] = pl[i][2];
        pf[i][3] = -gb * pl[i][0] + g * pl[i][3];
    }
    const double rs = sqrt(x1 * x2 * pr->s_lab);
    const double pa[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs};
    const double pb[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};
    event_tail(pr, chan, pf, pa, pb, x1, x2, factors, nf, ev);
}

/* ------------------------------------------------------------------------ */
/* Inverse mappings (section 2.1: every mapping is invertible, the density of */
/* a channel at given momenta is 1 / its Jacobian at the recovered point)     */
/* ------------------------------------------------------------------------ */

/* Inverse of G_nu: the r with orc_map_nu(r, ...) = x. */
double orc_unmap_nu(double x, double m2, double nu, double xmin, double xmax)
{
    if (nu == 0.0) return (x - xmin) / (xmax - xmin);
    if (nu == 1.0) {
        double lmax = log(xmax - m2), lmin = log(xmin - m2);
        return (log(x - m2) - lmin) / (lmax - lmin);
    }
    double e = 1.0 - nu;
    double A = pow(xmax - m2, e), B = pow(xmin - m2, e);
    return (pow(x - m2, e) - B) / (A - B);
}

/* Inverse of G_BW. */
double orc_unmap_bw(double x, double m, double w, double xmin, double xmax)
{
    double m2 = m * m, mw = m * w;
    double u1 = atan((xmin - m2) / mw), u2 = atan((xmax - m2) / mw);
    return (atan((x - m2) / mw) - u1) / (u2 - u1);
}

static double unmap_invariant(double x, double m, double w, double nu, double reg_a, double xmin, double xmax)
{
    if (w > 0.0) return orc_unmap_bw(x, m, w, xmin, xmax);
    double m2 = (m == 0.0) ? -reg_a : m * m;
    return orc_unmap_nu(x, m2, nu, xmin, xmax);
}

/* Inverse VEGAS map: the y whose image under orc_vegas_map is r (the bin
 * with e_i <= r < e_{i+1}, linear inside it). */
double orc_vegas_unmap(double r, const double* edges, int32_t nb)
{
    int32_t lo = 0, hi = nb - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) / 2;
        if (edges[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    double wdt = edges[lo + 1] - edges[lo];
    double t = wdt > 0.0 ? (r - edges[lo]) / wdt : 0.0;
    return (lo + t) / nb;
}

/* Azimuth of (x, y) as a fraction of a turn in [0, 1). */
static double turn_fraction(double x, double y)
{
    double f = atan2(y, x) / (2.0 * ORC_PI);
    return f < 0.0 ? f + 1.0 : f;
}

/* Inverse of the Chili generator (section 2.4), from the lab-frame momenta
 * of the final state: per particle but the last, p_T^2 -> r by inverting
 * eq. chili_pt_withcut (or p_T -> r by inverting eq. chili_pt_nocut), the
 * rapidity asinh(p_z / m_T) -> r within +-y_max(m_T), the azimuth measured
 * from the recoil direction of the particles before it -> r; then the last
 * particle's rapidity within its range.  Returns the number of dimensions
 * written. */
static int32_t inverse_chili(const orc_process* pr, double pl[][4], double* r)
{
    const int32_t n = pr->n_final;
    const double sq = sqrt(pr->s_lab), ptmax = 0.5 * sq;
    double q[ORC_MAX_FINAL][4];
    for (int32_t i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c) q[i][c] = pl[i + 2][c];
#ifdef ORC_LIBM_NUDGE
    for (int32_t i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c)
            if (q[i][c] != 0.0)
                q[i][c] = nextafter(q[i][c], ((i + c + (ORC_LIBM_NUDGE > 0)) & 1) ? INFINITY : -INFINITY);
#endif
    double sx = 0.0, sy = 0.0, ep = 0.0, em = 0.0;
    int32_t k = 0;
    for (int32_t i = 0; i < n - 1; ++i) {
        const double m = pr->mass[i];
        const double px = q[i][1], py = q[i][2], pz = q[i][3];
        const double pt2 = px * px + py * py;
        if (pr->pt_min > 0.0) {
            const double a = 1.0 / (ptmax * ptmax), b = 1.0 / (pr->pt_min * pr->pt_min);
            r[k++] = (b - 1.0 / pt2) / (b - a);
        } else {
            const double lam = m > 0.0 ? m : 1.0;
            const double pt = sqrt(pt2);
            r[k++] = pt * (2.0 * lam + ptmax) / (ptmax * (2.0 * lam + pt));
        }
        const double mt = sqrt(pt2 + m * m);
        const double z = sq / (2.0 * mt);
        const double ymax = log(z + sqrt(z * z - 1.0));
        const double yv = asinh(pz / mt);
        r[k++] = 0.5 * (yv / ymax + 1.0);
        /* azimuth relative to the recoil direction (-sx, -sy); +x for the first */
        const double ux = i == 0 ? 1.0 : -sx, uy = i == 0 ? 0.0 : -sy;
        r[k++] = turn_fraction(ux * px + uy * py, ux * py - uy * px);
        sx += px;
        sy += py;
        ep += mt * exp(yv);
        em += mt * exp(-yv);
    }
    {
        const int32_t i = n - 1;
        const double m = pr->mass[i];
        const double mt = sqrt(sx * sx + sy * sy + m * m);
        const double ylo = -log((sq - em) / mt), yhi = log((sq - ep) / mt);
        const double yv = asinh(q[i][3] / mt);
        r[k++] = (yv - ylo) / (yhi - ylo);
    }
    return k;
}

static void node_momentum(const orc_channel* ch, int32_t j, double pf[][4], double mom[][4])
{
    if (ch->kind[j] == ORC_LEAF) {
        memcpy(mom[j], pf[ch->particle[j]], sizeof mom[j]);
        return;
    }
    for (int c = 0; c < 4; ++c) mom[j][c] = 0.0;
    for (int32_t q = 0; q < ch->child_count[j]; ++q) {
        int32_t kid = ch->children[ch->child_start[j] + q];
        node_momentum(ch, kid, pf, mom);
        for (int c = 0; c < 4; ++c) mom[j][c] += mom[kid][c];
    }
}

/* The random numbers r (before VEGAS) that the channel's chain maps to the
 * given lab-frame momenta pl [n_final + 2][4] and momentum fractions: every
 * step of event() undone in its order.  Returns the number of dimensions. */
static int32_t inverse_event(const orc_process* pr, const orc_channel* ch, double pl[][4], double x1, double x2,
                             double* r)
{
    const int32_t n = pr->n_final;
    /* (8) undo the beam boost: (E, p_z) -> (g E - gb p_z, -gb E + g p_z) */
    double g = 1.0, gb = 0.0;
    if (pr->hadronic) {
        double sq = sqrt(x1 * x2);
        g = (x1 + x2) / (2.0 * sq);
        gb = (x1 - x2) / (2.0 * sq);
    }
    double pf[ORC_MAX_FINAL][4];
    for (int32_t i = 0; i < n; ++i) {
        const double* q = pl[i + 2];
        pf[i][0] = g * q[0] - gb * q[3];
        pf[i][1] = q[1];
        pf[i][2] = q[2];
        pf[i][3] = -gb * q[0] + g * q[3];
    }
#ifdef ORC_LIBM_NUDGE
    /* perturbation builds: the input momenta moved by one ulp as well */
    for (int32_t i = 0; i < n; ++i)
        for (int c = 0; c < 4; ++c)
            if (pf[i][c] != 0.0)
                pf[i][c] = nextafter(pf[i][c], ((i + c + (ORC_LIBM_NUDGE > 0)) & 1) ? INFINITY : -INFINITY);
#endif
    double mom[ORC_MAX_NODES][4];
    const int32_t root = ch->root;
    node_momentum(ch, root, pf, mom);

    double s[ORC_MAX_NODES];
    int32_t sampled[ORC_MAX_NODES];
    for (int32_t j = 0; j < ch->n_nodes; ++j) {
        s[j] = 0.0;
        sampled[j] = 0;
    }
    int32_t k = 0;

    /* (1) s-hat = x1 x2 s_lab */
    double shat;
    if (pr->hadronic) {
        double m = 0.0, w = 0.0, nu = pr->nu;
        if (ch->kind[root] == ORC_CLUSTER) {
            m = ch->mass[root];
            w = ch->width[root];
            nu = ch->nu[root];
        }
        double lo = pr->shat_min;
        double msum = 0.0;
        for (int32_t i = 0; i < n; ++i) msum += pr->mass[i];
        if (msum * msum > lo) lo = msum * msum;
        shat = x1 * x2 * pr->s_lab;
        r[k++] = unmap_invariant(shat, m, w, nu, pr->reg_a, lo, pr->s_lab);
    } else {
        shat = pr->s_lab;
    }
    s[root] = shat;
    sampled[root] = 1;

    /* (2) time-like invariants of the clusters from their momenta */
    for (int32_t q = 0; q < ch->n_sorder; ++q) {
        int32_t i = ch->s_order[q];
        double mmin = 0.0;
        for (int32_t c = 0; c < ch->child_count[i]; ++c)
            mmin += node_m_min(ch, ch->children[ch->child_start[i] + c], sampled, s);
        double mmax = node_m_max(ch, i, sampled, s);
        s[i] = mdot(mom[i], mom[i]);
        if (ch->rambo && ch->rambo[i] > 0)
            r[k++] = unmap_rambo(s[i], ch->rambo[i], mmin * mmin, mmax * mmax);
        else
            r[k++] = unmap_invariant(s[i], ch->mass[i], ch->width[i], ch->nu[i], pr->reg_a, mmin * mmin, mmax * mmax);
        sampled[i] = 1;
    }

    /* (3) t-channel order and the invariants of the remaining clusters */
    int32_t kappa = 0;
    int32_t sigma[ORC_MAX_FINAL + 1];
    int32_t from_a[ORC_MAX_FINAL + 1];
    double st[ORC_MAX_FINAL + 1];
    if (ch->kind[root] == ORC_TNODE) {
        kappa = ch->child_count[root] - 1;
        const int32_t* legs = ch->children + ch->child_start[root];
        int32_t lo = 0, hi = kappa;
        for (int32_t i = 1; i < kappa; ++i) {
            if (ch->t_order[i - 1] == 'A') {
                sigma[i] = legs[lo++];
                from_a[i] = 1;
            } else {
                sigma[i] = legs[hi--];
                from_a[i] = 0;
            }
        }
        sigma[kappa] = legs[lo];
        sigma[kappa + 1] = legs[hi];
        st[0] = shat;
        for (int32_t i = 1; i < kappa; ++i) {
            double msum = 0.0;
            for (int32_t j = i + 1; j <= kappa + 1; ++j) msum += node_m_min(ch, sigma[j], sampled, s);
            double mi = node_m_min(ch, sigma[i], sampled, s);
            double dm = sqrt(st[i - 1]) - mi;
            double Q[4] = {0.0, 0.0, 0.0, 0.0};
            for (int32_t j = i + 1; j <= kappa + 1; ++j)
                for (int c = 0; c < 4; ++c) Q[c] += mom[sigma[j]][c];
            st[i] = mdot(Q, Q);
            r[k++] = unmap_invariant(st[i], 0.0, 0.0, pr->nu, pr->reg_a, msum * msum, dm * dm);
        }
    }

    /* (4) x1 = tau^r */
    if (pr->hadronic) r[k++] = log(x1) / log(shat / pr->s_lab);

    double rs = sqrt(shat);
    double pa[4] = {0.5 * rs, 0.0, 0.0, 0.5 * rs};
    double pb[4] = {0.5 * rs, 0.0, 0.0, -0.5 * rs};

    /* (6) 2->2 blocks: |t| = -(p_A - p_1)^2, and the azimuth of p_1 about the
     *     direction of p_A in the rest frame of P = p_A + p_B */
    if (ch->kind[root] == ORC_TNODE) {
        double pA[4], pB[4];
        memcpy(pA, pa, sizeof pA);
        memcpy(pB, pb, sizeof pB);
        double ma2 = 0.0, mb2 = 0.0;
        for (int32_t i = 1; i <= kappa; ++i) {
            double m1, m2;
            if (i == kappa) {
                m1 = node_m_min(ch, sigma[kappa], sampled, s);
                m2 = node_m_min(ch, sigma[kappa + 1], sampled, s);
            } else if (from_a[i]) {
                m1 = node_m_min(ch, sigma[i], sampled, s);
                m2 = sqrt(st[i]);
            } else {
                m1 = sqrt(st[i]);
                m2 = node_m_min(ch, sigma[i], sampled, s);
            }
            double P[4] = {pA[0] + pB[0], pA[1] + pB[1], pA[2] + pB[2], pA[3] + pB[3]};
            double p1[4], p2[4];
            if (i == kappa || from_a[i]) {
                memcpy(p1, mom[sigma[i]], sizeof p1);
                for (int c = 0; c < 4; ++c) p2[c] = P[c] - p1[c];
            } else {
                memcpy(p2, mom[sigma[i]], sizeof p2);
                for (int c = 0; c < 4; ++c) p1[c] = P[c] - p2[c];
            }
            double d[4] = {pA[0] - p1[0], pA[1] - p1[1], pA[2] - p1[2], pA[3] - p1[3]};
            double abst = -mdot(d, d);
            if (ch->st && i >= 2) {
                double rs_, rt_;
                orc_two_to_two_st_inverse(pA, pB, mom[sigma[i - 1]], st[i - 1], ma2, mb2, m1, m2, p1, pr->nu,
                                          pr->reg_a, &rs_, &rt_);
                r[k++] = rs_;
                r[k++] = rt_;
                if (i < kappa) {
                    if (from_a[i]) {
                        for (int c = 0; c < 4; ++c) pA[c] -= p1[c];
                        ma2 = -abst;
                    } else {
                        for (int c = 0; c < 4; ++c) pB[c] -= p2[c];
                        mb2 = -abst;
                    }
                }
                continue;
            }
            double tmin, tmax;
            orc_t_range(st[i - 1], ma2, mb2, m1, m2, &tmin, &tmax);
            double m0 = sqrt(st[i - 1]);
            double Pbar[4] = {P[0], -P[1], -P[2], -P[3]};
            double pAr[4], k1[4];
            orc_boost(Pbar, m0, pA, pAr);
            orc_boost(Pbar, m0, p1, k1);
            double len = sqrt(pAr[1] * pAr[1] + pAr[2] * pAr[2] + pAr[3] * pAr[3]);
            double nx = pAr[1] / len, ny = pAr[2] / len, nz = pAr[3] / len;
            double sn = sqrt(nx * nx + ny * ny);
            double cp = 1.0, sp = 0.0;
            if (sn > 0.0) {
                cp = nx / sn;
                sp = ny / sn;
            }
            /* R(phi_A, theta_A)^-1 = R_y(-theta_A) R_z(-phi_A) */
            double x = k1[1] * cp + k1[2] * sp, y = -k1[1] * sp + k1[2] * cp, z = k1[3];
            double vx = x * nz - z * sn;
            double vy = y;
            r[k++] = turn_fraction(vx, vy);
            r[k++] = orc_unmap_nu(abst, -pr->reg_a, pr->nu, tmin, tmax);
            if (i < kappa) {
                if (from_a[i]) {
                    for (int c = 0; c < 4; ++c) pA[c] -= p1[c];
                    ma2 = -abst;
                } else {
                    for (int c = 0; c < 4; ++c) pB[c] -= p2[c];
                    mb2 = -abst;
                }
            }
        }
    } else {
        mom[root][0] = rs;
        mom[root][1] = mom[root][2] = mom[root][3] = 0.0;
    }

    /* (7) decays: angles of the first child in the rest frame of its parent */
    for (int32_t q = 0; q < ch->n_dec; ++q) {
        int32_t c = ch->dec_order[q];
        int32_t c0 = ch->children[ch->child_start[c]];
        double m0 = sqrt(s[c]);
        double Pbar[4] = {mom[c][0], -mom[c][1], -mom[c][2], -mom[c][3]};
        double kk[4];
        orc_boost(Pbar, m0, mom[c0], kk);
        if (ch->child_count[c] == 3) {
            /* 1 -> 3 decay (section 2.2.6): E1, E2 and the angles of p1 and of
             * p2 about p1 in the rest frame of the parent */
            int32_t c1 = ch->children[ch->child_start[c] + 1], c2 = ch->children[ch->child_start[c] + 2];
            double m1 = node_m_min(ch, c0, sampled, s), m2 = node_m_min(ch, c1, sampled, s);
            double m3 = node_m_min(ch, c2, sampled, s);
            double k2[4];
            orc_boost(Pbar, m0, mom[c1], k2);
            const double e1 = kk[0], e2 = k2[0];
            const double w1 = (m0 - m1 - (m2 + m3)) * (m0 - m1 + (m2 + m3)) / (2.0 * m0);
            r[k++] = (e1 - m1) / w1;
            const double q1sq = e1 * e1 - m1 * m1;
            const double dl = 2.0 * m0 * (0.5 * m0 - e1) + m1 * m1;
            const double d23 = m2 * m2 - m3 * m3;
            const double root = sqrt(fmax(0.0, q1sq * ((dl + d23) * (dl + d23) - 4.0 * m2 * m2 * dl)));
            const double e2min = ((m0 - e1) * (dl + d23) - root) / (2.0 * dl);
            r[k++] = (e2 - e2min) / (root / dl);
            const double len = sqrt(kk[1] * kk[1] + kk[2] * kk[2] + kk[3] * kk[3]);
            const double ux = kk[1] / len, uy = kk[2] / len, uz = kk[3] / len;
            r[k++] = turn_fraction(ux, uy);
            r[k++] = 0.5 * (uz + 1.0);
            /* p2 in the frame where p1 is along z: R(phi, theta)^-1 =
             * R_y(-theta) R_z(-phi) */
            const double st = sqrt(ux * ux + uy * uy);
            const double cp = st > 0.0 ? ux / st : 1.0, sp = st > 0.0 ? uy / st : 0.0;
            const double ax = cp * k2[1] + sp * k2[2], ay = -sp * k2[1] + cp * k2[2], az = k2[3];
            const double bx = uz * ax - st * az, by = ay;
            r[k++] = turn_fraction(bx, by);
            continue;
        }
        double len = sqrt(kk[1] * kk[1] + kk[2] * kk[2] + kk[3] * kk[3]);
        r[k++] = turn_fraction(kk[1], kk[2]);
        r[k++] = 0.5 * (kk[3] / len + 1.0);
    }
    return k;
}

/* Inverse map of n events of one channel: lab-frame momenta p
 * [4][n_final+2][n] and x1x2 [2][n] (hadronic; NULL otherwise) -> the
 * uniforms y [dims][n] (through the inverse VEGAS grid when grid is given),
 * and jac [n] = the forward Jacobian at y (the channel density is 1/jac).
 * Returns 0, or -1 on invalid sizes. */
int orc_inverse(const orc_process* pr, const orc_channel* ch, int32_t chan, int32_t dims, int64_t n,
                const double* p, const double* x1x2, const double* grid, int32_t nb, double* y, double* jac,
                int32_t nthreads)
{
    if (dims > ORC_MAX_DIMS || pr->n_final > ORC_MAX_FINAL || ch->n_nodes > ORC_MAX_NODES) return -1;
    const int32_t np = pr->n_final + 2;
    int bad = 0;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1) reduction(| : bad)
    for (int64_t e = 0; e < n; ++e) {
        double pl[ORC_MAX_FINAL + 2][4];
        for (int32_t i = 0; i < np; ++i)
            for (int c = 0; c < 4; ++c) pl[i][c] = p[((size_t)c * np + i) * n + e];
        double x1 = 1.0, x2 = 1.0;
        if (pr->hadronic) {
            x1 = x1x2[e];
            x2 = x1x2[n + e];
        }
        double r[ORC_MAX_DIMS], ye[ORC_MAX_DIMS];
        int32_t k = ch->chili ? inverse_chili(pr, pl, r) : inverse_event(pr, ch, pl, x1, x2, r);
        if (k < 0) {
            bad = 1;
            continue;
        }
        if (k != dims) {
            bad = 1;
            continue;
        }
        int outside = 0;
        for (int32_t q = 0; q < dims; ++q)
            if (!(r[q] >= -ORC_SUPPORT_MARGIN && r[q] <= 1.0 + ORC_SUPPORT_MARGIN)) outside = 1;
        if (outside) {
            /* not in the channel's image: no uniforms map there, density 0 */
            for (int32_t q = 0; q < dims; ++q) y[(size_t)q * n + e] = NAN;
            if (jac) jac[e] = 0.0;
            continue;
        }
        for (int32_t q = 0; q < dims; ++q)
            ye[q] = grid ? orc_vegas_unmap(r[q], grid + (size_t)q * (nb + 1), nb) : r[q];
        for (int32_t q = 0; q < dims; ++q) y[(size_t)q * n + e] = ye[q];
        if (jac) {
            orc_event ev;
            event(pr, ch, chan, ye, dims, grid, nb, &ev);
            jac[e] = ev.jac;
        }
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Batched entry point                                                       */
/* ------------------------------------------------------------------------ */

/* Map n events of one channel.  y: [dims][n] uniforms before VEGAS; grid:
 * [dims][nb+1] edges or NULL.  Outputs (any may be NULL): p [4][n_final+2][n],
 * x1x2 [2][n], jac [n], w [n], alpha [n], f [n], inv [n_nodes][n],
 * tabs [kappa][n] (|t| of each 2->2 block).
 * Returns 0, or -1 on invalid sizes. */
int orc_map(const orc_process* pr, const orc_channel* ch, int32_t chan, int32_t dims, int64_t n,
            const double* y, const double* grid, int32_t nb, double* p, double* x1x2, double* jac,
            double* w, double* alpha, double* f, double* inv, double* tabs, int32_t nthreads)
{
    if (dims > ORC_MAX_DIMS || pr->n_final > ORC_MAX_FINAL || ch->n_nodes > ORC_MAX_NODES) return -1;
    const int32_t np = pr->n_final + 2;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t e = 0; e < n; ++e) {
        double ye[ORC_MAX_DIMS];
        for (int32_t k = 0; k < dims; ++k) ye[k] = y[(size_t)k * n + e];
        orc_event ev;
        event(pr, ch, chan, ye, dims, grid, nb, &ev);
        if (p)
            for (int32_t i = 0; i < np; ++i)
                for (int c = 0; c < 4; ++c) p[((size_t)c * np + i) * n + e] = ev.p[i][c];
        if (x1x2) {
            x1x2[e] = ev.x1;
            x1x2[n + e] = ev.x2;
        }
        if (jac) jac[e] = ev.jac;
        if (w) w[e] = ev.w;
        if (alpha) alpha[e] = ev.alpha;
        if (f) f[e] = ev.f;
        if (inv)
            for (int32_t j = 0; j < ch->n_nodes; ++j) inv[(size_t)j * n + e] = ev.inv[j];
        if (tabs && ch->n_nodes > 0 && ch->kind[ch->root] == ORC_TNODE)
            for (int32_t j = 0; j < ch->child_count[ch->root] - 1; ++j) tabs[(size_t)j * n + e] = ev.tabs[j];
    }
    return 0;
}

/* Weight of given events: w = alpha_c f jac from lab-frame momenta p
 * [4][n_final+2][n] (incoming a, b first), x1x2 [2][n] (hadronic) and jac [n]
 * (events with jac = 0 get w = 0).  alpha [n] may be NULL. */
int orc_weight(const orc_process* pr, int32_t chan, int64_t n, const double* p, const double* x1x2,
               const double* jac, double* w, double* alpha, int32_t nthreads)
{
    if (pr->n_final > ORC_MAX_FINAL) return -1;
    const int32_t np = pr->n_final + 2;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int64_t e = 0; e < n; ++e) {
        double pf[ORC_MAX_FINAL][4], pa[4];
        for (int c = 0; c < 4; ++c) {
            pa[c] = p[((size_t)c * np + 0) * n + e];
            for (int32_t i = 0; i < pr->n_final; ++i) pf[i][c] = p[((size_t)c * np + i + 2) * n + e];
        }
#ifdef ORC_LIBM_NUDGE
        for (int32_t i = 0; i < pr->n_final; ++i)
            for (int c = 0; c < 4; ++c)
                if (pf[i][c] != 0.0)
                    pf[i][c] = nextafter(pf[i][c], ((i + c + (ORC_LIBM_NUDGE > 0)) & 1) ? INFINITY : -INFINITY);
#endif
        double x1 = 1.0, x2 = 1.0, a = 0.0, f = 0.0;
        if (pr->hadronic) {
            x1 = x1x2[e];
            x2 = x1x2[n + e];
        }
        if (jac[e] != 0.0) f = integrand(pr, chan, pf, pa, x1, x2, &a);
        w[e] = a * f * jac[e];
        if (alpha) alpha[e] = a;
    }
    return 0;
}

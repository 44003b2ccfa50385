// Per-event phase-space chain on gfx950: one thread per event, every lane of
// a wave in the same channel.  Channel tables are read with scalar loads;
// the per-event momentum slots and invariants live in small private arrays
// indexed only by wave-uniform values, which the compiler keeps in VGPRs
// (indexed with s_set_gpr_idx) instead of scratch.
//
// Steps follow section 2.2 of arXiv:2602.06895: s-hat (eqs. prop_stable_nu /
// prop_massive), time-like invariants with s-/t-channel bounds, the PDF
// convolution (eq. pdf_sampling), the chain of (phi, t) 2->2 blocks (eqs.
// t_invariant_theta, 2_to_2_mapping, ps2_phi_t), (phi, theta) decays (eq.
// ps2_phi_theta), the beam boost, the Jacobian product and the unphysical
// cut; then the integrand and the local channel weight (eq.
// multi-channel-mg).
#pragma once

#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#endif

#include "tables.h"

namespace msx {

constexpr double kPiD = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter-based generator.
// ---------------------------------------------------------------------------
// Full 64 x 64 -> 128-bit product from four 32 x 32 -> 64 partial products
// (each a v_mad_u64_u32 with the carry folded in), shared by both halves.
__device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    const uint64_t a0 = (uint32_t)a, a1 = a >> 32, b0 = (uint32_t)b, b1 = b >> 32;
    const uint64_t p00 = a0 * b0;
    const uint64_t mid = a0 * b1 + (p00 >> 32);           // < 2^64
    const uint64_t mid2 = a1 * b0 + (uint32_t)mid;        // < 2^64
    hi = a1 * b1 + (mid >> 32) + (mid2 >> 32);
    lo = (mid2 << 32) | (uint32_t)p00;
}

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3,
                                              uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t hi0, lo0, hi1, lo1;
        mul128(M0, c0, hi0, lo0);
        mul128(M1, c2, hi1, lo1);
        uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// 53 random bits -> (0, 1), never 0 or 1.
__device__ __forceinline__ double to_unit(uint64_t w) {
    return ((double)(w >> 11) + 0.5) * 0x1.0p-53;
}

// ---------------------------------------------------------------------------
// Small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double kallen(double x, double y, double z) {
    double d = x - y - z;
    return d * d - 4.0 * y * z;
}

__device__ __forceinline__ double ipow(double b, int n) {
    double b2 = b * b;
    switch (n) {
        case 1: return b;
        case 2: return b2;
        case 3: return b2 * b;
        case 4: return b2 * b2;
        case 5: return b2 * b2 * b;
        case 6: return b2 * b2 * b2;
        case 7: return b2 * b2 * b2 * b;
        default: return (b2 * b2) * (b2 * b2);
    }
}

// Map kinds compiled into a kernel (a launch picks the smallest set covering
// its channels; paths not compiled in cost no registers).
enum : int {
    KIND_POW_INT = 1,  // power law with 1/(1 - nu) an integer (k-th roots)
    KIND_POW = 2,      // general power law (pow)
    KIND_LOG = 4,      // nu = 1
    KIND_FLAT = 8,     // nu = 0
    KIND_BW = 16,      // Breit-Wigner
    KIND_RAMBO = 32,   // FastRambo cluster masses
    KINDS_ALL = 63,    // every tree-channel map kind
    KIND_CHILI = 64,   // Chili channels (compiled only for processes that use them)
    KIND_DEC3 = 128,   // 1 -> 3 decays (likewise)
    KIND_ST = 256      // (s~, t) blocks in the t-channel chain (likewise)
};

// Precision of the well-conditioned transcendentals (power laws, exp, log,
// angles).  MIX = false: FP64 throughout.  MIX = true: these are evaluated in
// FP32 on the FP64 argument rounded to float and widened back; everything
// whose rounding is amplified -- differences near threshold (Kallen
// functions, x - m^2, the t range, the s-channel mass bounds, the difference
// of the power-law endpoints), square roots of invariants, the momentum
// fractions x1, x2 (the PDFs take 1 - x), the Breit-Wigner arctangent /
// tangent (ill-conditioned off resonance), the boosts and the Jacobian
// product -- stays FP64.
template <bool MIX>
__device__ __forceinline__ double t_exp(double x) {
    return MIX ? (double)expf((float)x) : exp(x);
}
template <bool MIX>
__device__ __forceinline__ double t_log(double x) {
    return MIX ? (double)logf((float)x) : log(x);
}
template <bool MIX>
__device__ __forceinline__ double t_pow(double x, double e) {
    return MIX ? (double)powf((float)x, (float)e) : pow(x, e);
}
template <bool MIX>
__device__ __forceinline__ void t_sincospi(double x, double* s, double* c) {
    if (MIX) {
        float sf, cf;
        sincospif((float)x, &sf, &cf);
        *s = sf;
        *c = cf;
    } else {
        sincospi(x, s, c);
    }
}

// x^(1/k) for x >= 0 and integer k in 2..8 (inv_k = 1/k): an FP32 estimate
// of z = x^(-1/k) refined by two Newton steps on z^k x = 1, which need no
// division (z += z (1 - x z^k) / k), then x^(1/k) = x z^(k-1) (error a few
// ulp).  Outside the FP32 range the exponent is split off first.
template <bool MIX>
__device__ __forceinline__ double kth_root(double x, int k, double inv_k) {
    if (!(x > 0.0)) return x == 0.0 ? 0.0 : __builtin_nan("");
    if (MIX) return (double)exp2f(log2f((float)x) * (float)inv_k);
    int q = 0;
    double g = x;
    if (!(x > 1e-30 && x < 1e30)) {
        int ex;
        const double f = frexp(x, &ex);  // x = f 2^ex, f in [0.5, 1)
        q = ex >= 0 ? ex / k : -((-ex + k - 1) / k);
        g = ldexp(f, ex - q * k);  // in [0.5, 2^k)
    }
    double z = (double)exp2f(-log2f((float)g) * (float)inv_k);
#pragma unroll
    for (int it = 0; it < 2; ++it) z = fma(z * inv_k, fma(-g, ipow(z, k), 1.0), z);
    const double y = g * ipow(z, k - 1);
    return q ? ldexp(y, q) : y;
}

// (x - m2)^e for the power-law maps: a k-th root when e = 1/k.
template <int KINDS, bool MIX>
__device__ __forceinline__ double pow_e(const MapParams& p, double x) {
    if (!(KINDS & KIND_POW)) return kth_root<MIX>(x, p.int_pow, p.e);
    return p.int_pow ? kth_root<MIX>(x, p.int_pow, p.e) : t_pow<MIX>(x, p.e);
}

// b^n for an integer n >= 1 (square and multiply).
__device__ __forceinline__ double ipow_any(double b, int n) {
    double r = 1.0;
    while (n) {
        if (n & 1) r *= b;
        b *= b;
        n >>= 1;
    }
    return r;
}

// Power-law core: b = r A + (1 - r) B, x - m^2 = b^(1/e), and
// J = (A - B) (x - m^2)^nu / e with (x - m^2)^nu = (x - m^2) / b.
template <int KINDS, bool MIX>
__device__ __forceinline__ double pow_core(const MapParams& p, double A, double B, double r, double& jac) {
    double b = r * A + (1.0 - r) * B;
    double xm = (!(KINDS & KIND_POW) || p.int_pow) ? ipow(b, p.int_pow) : t_pow<MIX>(b, p.inv_e);
    jac = (A - B) * (xm / b) * p.inv_e;
    return xm + p.m2;
}

// G_nu / G_BW with bounds known only per event.
template <int KINDS, bool MIX>
__device__ __forceinline__ double map_dyn(const MapParams& p, double r, double xmin, double xmax, double& jac) {
    const int kind = p.kind;
    if ((KINDS & (KIND_POW | KIND_POW_INT)) && kind == MAP_POW) {
        if (MIX) {
            // A - B = B ((X / Y)^e - 1) = B expm1(e log1p((xmax - xmin) / Y)) with
            // Y = xmin - m2: no cancellation of two FP32 powers near threshold
            const double Y = xmin - p.m2;
            const double B = pow_e<KINDS, true>(p, Y);
            const float lr = log1pf((float)((xmax - xmin) / Y));
            const double AmB = B * (double)expm1f((float)p.e * lr);
            const double b = B + r * AmB;
            const double xm = (!(KINDS & KIND_POW) || p.int_pow) ? ipow(b, p.int_pow) : t_pow<true>(b, p.inv_e);
            jac = AmB * (xm / b) * p.inv_e;
            return xm + p.m2;
        }
        double A = pow_e<KINDS, MIX>(p, xmax - p.m2), B = pow_e<KINDS, MIX>(p, xmin - p.m2);
        return pow_core<KINDS, MIX>(p, A, B, r, jac);
    }
    if ((KINDS & KIND_BW) && kind == MAP_BW) {
        double u1 = atan((xmin - p.m2) / p.mw), u2 = atan((xmax - p.m2) / p.mw);
        double d = p.mw * tan(u1 + (u2 - u1) * r);
        jac = (u2 - u1) * (d * d + p.mw * p.mw) / p.mw;
        return d + p.m2;
    }
    if ((KINDS & KIND_RAMBO) && kind == MAP_RAMBO) {
        // FastRambo (section 2.2.9): y = G_RQF^-1(r, c_k) in closed form,
        // u = y^(1/2k), M = mu + u (M_max - mu) with mu = sqrt(xmin) (the
        // cluster's masses) and M_max = sqrt(xmax); massless: M = u M_parent.
        // dM^2/dr = 2 M (M_max - mu) u / (2 k y g_RQF(y, c_k)).  FP64.
        const double c = p.mw;
        const double b = c - (c - 2.0) * r;
        const double y = 2.0 * r / (b + sqrt(b * b + 4.0 * r * (1.0 - b)));
        const double u = sqrt(p.int_pow == 1 ? y : kth_root<false>(y, p.int_pow, p.e));  // y^(1/2k), k <= 7
        const double lo = sqrt(xmin), span = sqrt(xmax) - lo;
        const double m = lo + u * span;
        const double om = y * (1.0 - y);
        const double den = 1.0 + (c - 2.0) * om;
        const double g = (2.0 * om + c * (1.0 - y) * (1.0 - y)) / (den * den);
        jac = 2.0 * m * span * u * (0.5 * p.e) / (y * g);
        return m * m;
    }
    if ((KINDS & KIND_LOG) && kind == MAP_LOG) {
        double lmax = t_log<MIX>(xmax - p.m2), lmin = t_log<MIX>(xmin - p.m2);
        double xm = t_exp<MIX>(r * lmax + (1.0 - r) * lmin);
        jac = xm * (lmax - lmin);
        return xm + p.m2;
    }
    jac = xmax - xmin;
    return xmin + (xmax - xmin) * r;
}

// G_nu / G_BW with precomputed static constants (s-hat).
template <int KINDS, bool MIX>
__device__ __forceinline__ double map_static(const InvSpec& iv, double r, double& jac) {
    const MapParams& p = iv.map;
    const int kind = p.kind;
    if ((KINDS & (KIND_POW | KIND_POW_INT)) && kind == MAP_POW) return pow_core<KINDS, MIX>(p, iv.A, iv.B, r, jac);
    if ((KINDS & KIND_BW) && kind == MAP_BW) {
        double u2 = iv.A, u1 = iv.B;
        double d = p.mw * tan(u1 + (u2 - u1) * r);
        jac = (u2 - u1) * (d * d + p.mw * p.mw) / p.mw;
        return d + p.m2;
    }
    if ((KINDS & KIND_LOG) && kind == MAP_LOG) {
        double lmax = iv.A, lmin = iv.B;
        double xm = t_exp<MIX>(r * lmax + (1.0 - r) * lmin);
        jac = xm * (lmax - lmin);
        return xm + p.m2;
    }
    jac = iv.xmax - iv.xmin;
    return iv.xmin + (iv.xmax - iv.xmin) * r;
}

// Inverses of the maps (FP64): the r that map_dyn / map_static send to x.
template <int KINDS>
__device__ __forceinline__ double unmap_dyn(const MapParams& p, double x, double xmin, double xmax) {
    const int kind = p.kind;
    if ((KINDS & (KIND_POW | KIND_POW_INT)) && kind == MAP_POW) {
        const double A = pow_e<KINDS, false>(p, xmax - p.m2), B = pow_e<KINDS, false>(p, xmin - p.m2);
        return (pow_e<KINDS, false>(p, x - p.m2) - B) / (A - B);
    }
    if ((KINDS & KIND_BW) && kind == MAP_BW) {
        const double u1 = atan((xmin - p.m2) / p.mw), u2 = atan((xmax - p.m2) / p.mw);
        return (atan((x - p.m2) / p.mw) - u1) / (u2 - u1);
    }
    if ((KINDS & KIND_RAMBO) && kind == MAP_RAMBO) {
        const double lo = sqrt(xmin);
        const double u = (sqrt(x) - lo) / (sqrt(xmax) - lo);
        const double y = ipow_any(u, 2 * p.int_pow), c = p.mw;
        return (y * y + c * y * (1.0 - y)) / (1.0 + (c - 2.0) * y * (1.0 - y));
    }
    if ((KINDS & KIND_LOG) && kind == MAP_LOG) {
        const double lmax = log(xmax - p.m2), lmin = log(xmin - p.m2);
        return (log(x - p.m2) - lmin) / (lmax - lmin);
    }
    return (x - xmin) / (xmax - xmin);
}

template <int KINDS>
__device__ __forceinline__ double unmap_static(const InvSpec& iv, double x) {
    const MapParams& p = iv.map;
    const int kind = p.kind;
    if ((KINDS & (KIND_POW | KIND_POW_INT)) && kind == MAP_POW)
        return (pow_e<KINDS, false>(p, x - p.m2) - iv.B) / (iv.A - iv.B);
    if ((KINDS & KIND_BW) && kind == MAP_BW) return (atan((x - p.m2) / p.mw) - iv.B) / (iv.A - iv.B);
    if ((KINDS & KIND_LOG) && kind == MAP_LOG) return (log(x - p.m2) - iv.B) / (iv.A - iv.B);
    return (x - iv.xmin) / (iv.xmax - iv.xmin);
}

// Azimuth of (x, y) as a fraction of a turn in [0, 1).
__device__ __forceinline__ double turn_fraction(double x, double y) {
    const double f = atan2(y, x) / (2.0 * kPiD);
    return f < 0.0 ? f + 1.0 : f;
}

// Inverse VEGAS map: the bin with e_i <= r < e_{i+1} by bisection, linear
// inside it.
__device__ __forceinline__ double vegas_unmap(double r, const double* __restrict__ g, int nb) {
    int lo = 0, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (g[mid] <= r) lo = mid;
        else hi = mid - 1;
    }
    const double wd = g[lo + 1] - g[lo];
    const double t = wd > 0.0 ? (r - g[lo]) / wd : 0.0;
    return (lo + t) / nb;
}

// Sum of the final-state momenta in `set` (statically indexed arrays).
template <int NF>
__device__ __forceinline__ void sum_set(uint32_t set, const double (&FE)[NF], const double (&FX)[NF],
                                        const double (&FY)[NF], const double (&FZ)[NF], double& qe, double& qx,
                                        double& qy, double& qz) {
    qe = qx = qy = qz = 0.0;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        if (set & (1u << k)) {
            qe += FE[k];
            qx += FX[k];
            qy += FY[k];
            qz += FZ[k];
        }
    }
}

// Pure boost of k from the rest frame of P (mass m) into the frame of P,
// with inv_m = 1/m and inv_em = 1/(E_P + m) supplied (shared by the boosts of
// one operation).
__device__ __forceinline__ void boost_by(double Pe, double Px, double Py, double Pz, double inv_m, double inv_em,
                                         double& ke, double& kx, double& ky, double& kz) {
    double pk = Px * kx + Py * ky + Pz * kz;
    double e = (Pe * ke + pk) * inv_m;
    double c = (pk * inv_em + ke) * inv_m;
    ke = e;
    kx += c * Px;
    ky += c * Py;
    kz += c * Pz;
}

// ---------------------------------------------------------------------------
// Per-event state.  NS: momentum slots; the uniforms are held in two
// 16-entry arrays (dims <= 32).  All arrays are indexed by uniform values.
// ---------------------------------------------------------------------------
struct ChainOut {
    double shat, x1, x2, logtau, jac;
    bool ok;
};

// Register index of a slot code (codes >= 0 count from the bottom of the
// slot file, codes < 0 from the top).
template <int NS>
__device__ __forceinline__ int slot_index(int code) {
    return code >= 0 ? code : NS + code;
}

template <int NI>
__device__ __forceinline__ double src_mass(const MassSrc& ms, const double (&SQ)[NI]) {
    return ms.inv >= 0 ? SQ[ms.inv] : ms.m;
}

template <int NI>
__device__ __forceinline__ double masked_sum(uint32_t mask, const double (&SQ)[NI]) {
    double s = 0.0;
    while (mask) {
        int b = __builtin_ctz(mask);
        s += SQ[b];
        mask &= mask - 1;
    }
    return s;
}

// 1 -> 3 decay (section 2.2.6) in the rest frame of the parent (mass m0):
// E1 linear in [m1, E1max], E2 linear in [E2min, E2max] (the range of the
// two-body decay of p2 + p3, of mass^2 m0^2 - 2 m0 E1 + m1^2, seen from the
// parent's rest frame), p1 along R(phi, theta) z, p2 along R(phi, theta)
// R(beta, alpha) z with cos(alpha) fixed by momentum conservation, p3 the
// rest.  Random numbers (E1, E2, phi, theta, beta).  Returns the measure
// (1/8) dE1 dE2 dphi dbeta dcos(theta) = pi^2 (E1max - m1)(E2max - E2min).
// FP64 in both precisions.
__device__ __forceinline__ double three_body_rest(double m0, double m1, double m2, double m3, const double (&r)[5],
                                                  double (&k1)[4], double (&k2)[4], double (&k3)[4]) {
    // E1max - m1 = ((m0 - m1)^2 - (m2 + m3)^2) / (2 m0), factored (no
    // cancellation near threshold)
    const double w1 = (m0 - m1 - (m2 + m3)) * (m0 - m1 + (m2 + m3)) / (2.0 * m0);
    const double e1 = m1 + w1 * r[0];
    const double q1 = sqrt(fmax(0.0, e1 * e1 - m1 * m1));
    const double dl = 2.0 * m0 * (0.5 * m0 - e1) + m1 * m1;
    const double d23 = m2 * m2 - m3 * m3;
    const double root = sqrt(fmax(0.0, q1 * q1 * ((dl + d23) * (dl + d23) - 4.0 * m2 * m2 * dl)));
    // E2max - E2min = root / dl exactly (no difference of the range ends)
    const double e2min = ((m0 - e1) * (dl + d23) - root) / (2.0 * dl);
    const double w2 = root / dl;
    const double e2 = e2min + w2 * r[1];
    const double q2 = sqrt(fmax(0.0, e2 * e2 - m2 * m2));
    double ca = (2.0 * m0 * (0.5 * m0 - e1 - e2) + m1 * m1 + m2 * m2 + 2.0 * e1 * e2 - m3 * m3) / (2.0 * q1 * q2);
    ca = ca >= -1.0 ? fmin(ca, 1.0) : -1.0;  // rounding at the range ends (and 0/0)
    const double sa = sqrt((1.0 - ca) * (1.0 + ca));
    const double ct = 2.0 * r[3] - 1.0;
    const double st = sqrt((1.0 - ct) * (1.0 + ct));
    double sp, cp, sb, cb;
    sincos(2.0 * kPiD * r[2], &sp, &cp);
    sincos(2.0 * kPiD * r[4], &sb, &cb);
    // R(phi, theta) = R_z(phi) R_y(theta) on v = R(beta, alpha) z
    const double vx = cb * sa, vy = sb * sa, vz = ca;
    const double wx = ct * vx + st * vz, wy = vy, wz = -st * vx + ct * vz;
    k1[0] = e1;
    k1[1] = q1 * (cp * st);
    k1[2] = q1 * (sp * st);
    k1[3] = q1 * ct;
    k2[0] = e2;
    k2[1] = q2 * (cp * wx - sp * wy);
    k2[2] = q2 * (sp * wx + cp * wy);
    k2[3] = q2 * wz;
    k3[0] = m0 - e1 - e2;
    k3[1] = -k1[1] - k2[1];
    k3[2] = -k1[2] - k2[2];
    k3[3] = -k1[3] - k2[3];
    const double jac = kPiD * kPiD * w1 * w2;
    return jac > 0.0 ? jac : 0.0;
}

// The mapping chain.  next() returns the VEGAS-mapped random number of the
// next dimension (dimensions are consumed in order).  Leaves the final-state
// momenta in the partonic frame in the slots.
template <int NS, int NI, int KINDS, bool MIX, class Next>
__device__ __forceinline__ void run_chain(const ChannelTab* __restrict__ ct, double s_lab, Next& next,
                                          double (&E)[NS], double (&X)[NS], double (&Y)[NS], double (&Z)[NS],
                                          double (&S)[NI], double (&SQ)[NI], ChainOut& o) {
    double jac = ct->jac_const;
    const int hadronic = ct->hadronic;

    // (1) s-hat
    double shat;
    if (hadronic) {
        double j;
        shat = map_static<KINDS, MIX>(ct->inv[0], next(), j);
        jac *= j;
    } else {
        shat = s_lab;
    }
    S[0] = shat;
    SQ[0] = sqrt(shat);

    // (2) time-like invariants: bounds as linear forms in sqrt(s_j)
    const int n_inv = ct->n_inv;
    for (int i = 1; i < n_inv; ++i) {
        const InvSpec& iv = ct->inv[i];
        double mmin = iv.min_const + masked_sum(iv.min_mask, SQ);
        double mmax = SQ[iv.parent] - iv.max_const - masked_sum(iv.max_mask, SQ);
        double j;
        double s = map_dyn<KINDS, MIX>(iv.map, next(), mmin * mmin, mmax * mmax, j);
        jac *= j;
        S[i] = s;
        SQ[i] = sqrt(s);
    }

    // (3) momentum fractions x1 = tau^r, x2 = tau^(1-r), J = -log(tau)/s_lab
    double x1 = 1.0, x2 = 1.0, L = 0.0;
    if (hadronic) {
        double r = next();
        // FP64 in both precisions: the PDFs take 1 - x, which cancels for x -> 1
        L = log(shat / s_lab);
        x1 = exp(r * L);
        x2 = exp((1.0 - r) * L);
        jac *= -L / s_lab;
    }

    // (4) 2->2 blocks along the t-channel spine.  The block invariants are
    // the sampled ones: (p_A + p_B)^2 = s of the remaining cluster, p_A^2 and
    // p_B^2 = 0 or the t of the block that last updated the leg.
    const double h = 0.5 * SQ[0];
    double Ae = h, Ax = 0.0, Ay = 0.0, Az = h;   // p_A
    double Be = h, Bx = 0.0, By = 0.0, Bz = -h;  // p_B
    double ma2 = 0.0, mb2 = 0.0;
    // Both loops are unrolled so that every slot store has a constant index
    // (block b -> slots 2b, 2b+1; decay d -> NS-2-2d, NS-1-2d): a store with a
    // run-time index would turn the slot file into selects.
    const int n_blocks = ct->n_blocks;
#pragma unroll
    for (int bi = 0; bi < NS / 2; ++bi) {
        if (bi >= n_blocks) break;
        const BlockSpec& bs = ct->blk[bi];
        double m1 = src_mass(bs.m1, SQ), m2 = src_mass(bs.m2, SQ);
        double r_phi = next();
        double r_t = next();
        double Pe = Ae + Be, Px = Ax + Bx, Py = Ay + By, Pz = Az + Bz;
        double m0sq = S[bs.m0_inv];
        double m0 = SQ[bs.m0_inv];
        double m1s = m1 * m1, m2s = m2 * m2;
        double lam12 = kallen(m0sq, m1s, m2s), lamab = kallen(m0sq, ma2, mb2);
        double C = (m0sq + (m1s - m2s)) * (m0sq + (ma2 - mb2));
        double R = sqrt(lam12 * lamab);
        double inv2 = 1.0 / (2.0 * m0sq);
        // t at cos(theta) = -1 directly; the root at +1 from the product of
        // roots t+ t- = (m1^2-ma^2)(m2^2-mb^2) + (ma^2-mb^2-m1^2+m2^2)(ma^2 m2^2-m1^2 mb^2)/m0^2
        double t_minus = m1s + ma2 - (C + R) * inv2;
        double prod = (m1s - ma2) * (m2s - mb2) + (ma2 - mb2 - m1s + m2s) * (ma2 * m2s - m1s * mb2) / m0sq;
        double t_plus = (t_minus != 0.0) ? prod / t_minus : 0.0;
        double tmin = fmax(0.0, -t_plus);
        double tmax = -t_minus;
        double jt;
        double abst = map_dyn<KINDS, MIX>(bs.tmap, r_t, tmin, tmax, jt);
        double cth = (C - 2.0 * m0sq * (m1s + ma2 + abst)) / R;
        cth = fmin(1.0, fmax(-1.0, cth));
        double sth = sqrt((1.0 - cth) * (1.0 + cth));
        double sphi, cphi;
        double inv_2m0 = 1.0 / (2.0 * m0);
        double q = sqrt(lam12) * inv_2m0;
        double e1 = (m0sq + (m1s - m2s)) * inv_2m0;
        double e2 = (m0sq - (m1s - m2s)) * inv_2m0;
        // (s~, t) block (section 2.2.5): the azimuth about p_A comes from
        // s~ = (p1 + rec)^2 with rec the leg the previous block peeled,
        // measured from the plane of p_A and rec in the rest frame of P;
        // the half of [0, 1) that r_phi falls in gives the sign of sin(phi)
        const bool st_block = (KINDS & KIND_ST) && ct->st && bi > 0 && !bs.com;
        double jphi = 2.0 * kPiD;
        if (st_block) {
            const int prev_side = ct->blk[bi > 0 ? bi - 1 : 0].side;
            const int s1 = bi > 0 ? 2 * bi - 2 : 0, s2 = bi > 0 ? 2 * bi - 1 : 0;
            const double re = prev_side == 1 ? E[s2] : E[s1], rx0 = prev_side == 1 ? X[s2] : X[s1];
            const double ry0 = prev_side == 1 ? Y[s2] : Y[s1], rz0 = prev_side == 1 ? Z[s2] : Z[s1];
            const double Pe = Ae + Be, Px = Ax + Bx, Py = Ay + By, Pz = Az + Bz;
            const double i_m0 = 1.0 / m0, i_em = 1.0 / (Pe + m0);
            double ae = Ae, ax = Ax, ay = Ay, az = Az;
            boost_by(Pe, -Px, -Py, -Pz, i_m0, i_em, ae, ax, ay, az);
            double ce = re, cx = rx0, cy = ry0, cz = rz0;
            boost_by(Pe, -Px, -Py, -Pz, i_m0, i_em, ce, cx, cy, cz);
            (void)ce;
            const double inv_len = 1.0 / sqrt(ax * ax + ay * ay + az * az);
            const double nx = ax * inv_len, ny = ay * inv_len, nz = az * inv_len;
            const double snt = sqrt(nx * nx + ny * ny);
            double cp = 1.0, sp = 0.0;
            if (snt > 0.0) {
                const double ist = 1.0 / snt;
                cp = nx * ist;
                sp = ny * ist;
            }
            // the recoil's transverse direction with p_A along z:
            // R(phi_A, theta_A)^-1
            const double xr = cx * cp + cy * sp, yr = -cx * sp + cy * cp;
            const double u0 = xr * nz - cz * snt, u1 = yr;
            const double rperp = sqrt(u0 * u0 + u1 * u1);
            // s~ = A - B cos(phi) (A, B from the energies and angles of p1 and
            // rec) is uniform between A - B and A + B: s~ = (A - B) + 2 B u,
            // so cos(phi) = (A - s~) / B = 1 - 2 u, formed so without A
            // cancelling against s~
            const bool upper = r_phi >= 0.5;
            const double u = upper ? 2.0 * r_phi - 1.0 : 2.0 * r_phi;
            const double c = 1.0 - 2.0 * u;
            const double sn = (upper ? -2.0 : 2.0) * sqrt(u * (1.0 - u));
            const double ux = u0 / rperp, uy = u1 / rperp;
            cphi = ux * c - uy * sn;
            sphi = uy * c + ux * sn;
            // dphi / dr = 4 / |sin(phi)| on the two branches together
            jphi = 4.0 / fabs(sn);
        } else {
            t_sincospi<MIX>(2.0 * r_phi, &sphi, &cphi);
        }
        double vx = q * sth * cphi, vy = q * sth * sphi, vz = q * cth;
        double k1e = e1, k1x, k1y, k1z, k2e = e2, k2x, k2y, k2z;
        double inv_m0 = 0.0, inv_em = 0.0;
        if (bs.com) {
            // P at rest, p_A along +z: no rotation, no boost
            k1x = vx;
            k1y = vy;
            k1z = vz;
        } else {
            // direction of p_A in the rest frame of P, then R(phi_A, theta_A)
            inv_m0 = 1.0 / m0;
            inv_em = 1.0 / (Pe + m0);
            double ae = Ae, ax = Ax, ay = Ay, az = Az;
            boost_by(Pe, -Px, -Py, -Pz, inv_m0, inv_em, ae, ax, ay, az);
            double inv_len = 1.0 / sqrt(ax * ax + ay * ay + az * az);
            double nx = ax * inv_len, ny = ay * inv_len, nz = az * inv_len;
            double st = sqrt(nx * nx + ny * ny);
            double cp = 1.0, sp = 0.0;
            if (st > 0.0) {
                const double ist = 1.0 / st;
                cp = nx * ist;
                sp = ny * ist;
            }
            double rx = vx * nz + vz * st;
            double ry = vy;
            double rz = -vx * st + vz * nz;
            k1x = rx * cp - ry * sp;
            k1y = rx * sp + ry * cp;
            k1z = rz;
        }
        k2x = -k1x;
        k2y = -k1y;
        k2z = -k1z;
        if (!bs.com) {
            boost_by(Pe, Px, Py, Pz, inv_m0, inv_em, k1e, k1x, k1y, k1z);
            boost_by(Pe, Px, Py, Pz, inv_m0, inv_em, k2e, k2x, k2y, k2z);
        }
        jac *= jt * jphi / (4.0 * sqrt(lamab));
        // store both outputs and update the legs with uniform 0/1 factors:
        // leg next to A -> p_A -= p1, next to B -> p_B -= p2, last block -> neither
        E[2 * bi] = k1e;
        X[2 * bi] = k1x;
        Y[2 * bi] = k1y;
        Z[2 * bi] = k1z;
        E[2 * bi + 1] = k2e;
        X[2 * bi + 1] = k2x;
        Y[2 * bi + 1] = k2y;
        Z[2 * bi + 1] = k2z;
        const int side = bs.side;
        const double fa = side == 0 ? 1.0 : 0.0, fb = side == 1 ? 1.0 : 0.0;
        Ae -= fa * k1e;
        Ax -= fa * k1x;
        Ay -= fa * k1y;
        Az -= fa * k1z;
        Be -= fb * k2e;
        Bx -= fb * k2x;
        By -= fb * k2y;
        Bz -= fb * k2z;
        ma2 = side == 0 ? -abst : ma2;
        mb2 = side == 1 ? -abst : mb2;
    }

    // (5) (phi, theta) decays, parents before children
    const int n_dec = ct->n_decays;
#pragma unroll
    for (int di = 0; di < NS / 2; ++di) {
        if (di >= n_dec) break;
        const DecaySpec& ds = ct->dec[di];
        if (KINDS & KIND_DEC3) {
            if (ds.kind == 2) continue;  // the slots of the 1 -> 3 decay before
            if (ds.kind == 1) {
                const double m0 = SQ[ds.parent_inv];
                double rr[5];
#pragma unroll
                for (int q = 0; q < 5; ++q) rr[q] = next();
                double k1[4], k2[4], k3[4];
                jac *= three_body_rest(m0, src_mass(ds.m1, SQ), src_mass(ds.m2, SQ), src_mass(ds.m3, SQ), rr, k1,
                                       k2, k3);
                if (!ds.parent_rest) {
                    const int ps = slot_index<NS>(ds.parent_slot);
                    double Pe = E[ps], Px = X[ps], Py = Y[ps], Pz = Z[ps];
                    const double inv_m = 1.0 / m0, inv_em = 1.0 / (Pe + m0);
                    boost_by(Pe, Px, Py, Pz, inv_m, inv_em, k1[0], k1[1], k1[2], k1[3]);
                    boost_by(Pe, Px, Py, Pz, inv_m, inv_em, k2[0], k2[1], k2[2], k2[3]);
                    boost_by(Pe, Px, Py, Pz, inv_m, inv_em, k3[0], k3[1], k3[2], k3[3]);
                }
                // a 1 -> 3 decay is never the last entry (its pair follows),
                // so the third slot index is >= 0 whenever this runs
                const int s3 = NS - 4 - 2 * di >= 0 ? NS - 4 - 2 * di : 0;
                E[NS - 2 - 2 * di] = k1[0];
                X[NS - 2 - 2 * di] = k1[1];
                Y[NS - 2 - 2 * di] = k1[2];
                Z[NS - 2 - 2 * di] = k1[3];
                E[NS - 1 - 2 * di] = k2[0];
                X[NS - 1 - 2 * di] = k2[1];
                Y[NS - 1 - 2 * di] = k2[2];
                Z[NS - 1 - 2 * di] = k2[3];
                E[s3] = k3[0];
                X[s3] = k3[1];
                Y[s3] = k3[2];
                Z[s3] = k3[3];
                continue;
            }
        }
        double m0sq = S[ds.parent_inv];
        double m0 = SQ[ds.parent_inv];
        double m1 = src_mass(ds.m1, SQ), m2 = src_mass(ds.m2, SQ);
        double r_phi = next();
        double r_th = next();
        double m1s = m1 * m1, m2s = m2 * m2;
        double lam = kallen(m0sq, m1s, m2s);
        const double inv_m = 1.0 / m0;
        const double inv_2m0 = 0.5 * inv_m;
        double e1 = (m0sq + (m1s - m2s)) * inv_2m0;
        double e2 = (m0sq - (m1s - m2s)) * inv_2m0;
        double sl = sqrt(lam);
        double q = sl * inv_2m0;
        double cth = 2.0 * r_th - 1.0;
        double sth = sqrt((1.0 - cth) * (1.0 + cth));
        double sphi, cphi;
        t_sincospi<MIX>(2.0 * r_phi, &sphi, &cphi);
        double k1e = e1, k1x = q * sth * cphi, k1y = q * sth * sphi, k1z = q * cth;
        double k2e = e2, k2x = -k1x, k2y = -k1y, k2z = -k1z;
        if (!ds.parent_rest) {
            const int ps = slot_index<NS>(ds.parent_slot);
            double Pe = E[ps], Px = X[ps], Py = Y[ps], Pz = Z[ps];
            const double inv_em = 1.0 / (Pe + m0);
            boost_by(Pe, Px, Py, Pz, inv_m, inv_em, k1e, k1x, k1y, k1z);
            boost_by(Pe, Px, Py, Pz, inv_m, inv_em, k2e, k2x, k2y, k2z);
        }
        E[NS - 2 - 2 * di] = k1e;
        X[NS - 2 - 2 * di] = k1x;
        Y[NS - 2 - 2 * di] = k1y;
        Z[NS - 2 - 2 * di] = k1z;
        E[NS - 1 - 2 * di] = k2e;
        X[NS - 1 - 2 * di] = k2x;
        Y[NS - 1 - 2 * di] = k2y;
        Z[NS - 1 - 2 * di] = k2z;
        // two-body factor pi |p| / (2 m0) = pi sqrt(lambda) / (4 m0^2) ... as
        // sqrt(lambda) / (8 m0^2) times the 4 pi of the angles
        jac *= sl * (inv_m * inv_m) * (0.5 * kPiD);
    }

    o.shat = shat;
    o.x1 = x1;
    o.x2 = x2;
    o.logtau = L;
    o.jac = jac;
}

// Chili (section 2.4): every final-state particle but the last from
// (p_T, y, phi) in the lab frame -- p_T^2 by the 1/p_T^2 map between the
// process's p_T cut and sqrt(s_lab)/2 (eq. chili_pt_withcut), or without a
// cut the regulated map of eq. chili_pt_nocut with lambda = m (1 when
// massless); y uniform within +-y_max(m_T); phi uniform, measured from the
// direction of the current recoil -- then the last particle balances the
// transverse momentum and takes a rapidity uniform in the range the beam
// energy leaves, and x1,2 = E +- p_z summed / sqrt(s_lab).  The measure
// dx1 dx2 prod d^3p / 2E with the momentum delta becomes (2 pi)^(4-3n) /
// s_lab dy_n prod_(i<n) dp_T^2 dy dphi / 4 (the first factor is the
// channel's jac_const).  Particle k goes to slot k, boosted to the partonic
// frame so that the common tail boosts it back.  FP64 in both precisions.
template <int NS, class Next>
__device__ __forceinline__ void run_chili(const ChannelTab* __restrict__ ct, double s_lab, Next& next,
                                          double (&E)[NS], double (&X)[NS], double (&Y)[NS], double (&Z)[NS],
                                          ChainOut& o) {
    constexpr int NF = NS / 2 + 1;
    const int n = ct->n_final;
    const double sq = sqrt(s_lab), ptmax = 0.5 * sq;
    const double ptmin2 = ct->chili_ptmin2;
    double jac = ct->jac_const;
    double sx = 0.0, sy = 0.0, ep = 0.0, em = 0.0;
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NF - 1; ++i) {
        if (i >= n - 1) break;
        const double m = ct->chili_m[i];
        const double rp = next(), ryv = next(), rf = next();
        double pt2, jpt2;
        if (ptmin2 > 0.0) {
            const double a = 1.0 / (ptmax * ptmax), b = 1.0 / ptmin2;
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
        ok = ok && z > 1.0;
        const double ymax = ok ? log(z + sqrt(z * z - 1.0)) : 0.0;
        const double yv = ymax * (2.0 * ryv - 1.0);
        const double phi_rec = i == 0 ? 0.0 : atan2(-sy, -sx);
        double sphi, cphi;
        sincos(2.0 * kPiD * rf + phi_rec, &sphi, &cphi);
        const double pt = sqrt(pt2);
        // E +- p_z = m_T exp(+-y): the light-cone sums without cancellation
        const double lp = mt * exp(yv), lm = mt * exp(-yv);
        const double lx = pt * cphi, ly = pt * sphi;
        E[i] = 0.5 * (lp + lm);
        X[i] = lx;
        Y[i] = ly;
        Z[i] = 0.5 * (lp - lm);
        sx += lx;
        sy += ly;
        ep += lp;
        em += lm;
        jac *= jpt2 * (2.0 * ymax) * (2.0 * kPiD) / 4.0;
    }
    {
        const double m = ct->chili_m[n - 1];
        const double px = -sx, py = -sy;
        const double mt = sqrt(px * px + py * py + m * m);
        const double ylo = -log((sq - em) / mt), yhi = log((sq - ep) / mt);
        ok = ok && sq > ep && sq > em && yhi > ylo;
        const double rl = next();
        const double yv = ok ? ylo + (yhi - ylo) * rl : 0.0;
        const double lp = mt * exp(yv), lm = mt * exp(-yv);
        const double le = 0.5 * (lp + lm), lz = 0.5 * (lp - lm);
#pragma unroll
        for (int i = 0; i < NF; ++i)
            if (i == n - 1) {
                E[i] = le;
                X[i] = px;
                Y[i] = py;
                Z[i] = lz;
            }
        ep += lp;
        em += lm;
        jac *= ok ? (yhi - ylo) : 0.0;
    }
    double x1 = ep / sq, x2 = em / sq;
    if (!ok) x1 = x2 = 0.5;  // any values: the zero Jacobian cuts the event
    const double sqx = sqrt(x1 * x2);
    const double g = (x1 + x2) / (2.0 * sqx), gb = (x1 - x2) / (2.0 * sqx);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        if (i >= n) break;
        const double le = E[i], lz = Z[i];
        E[i] = g * le - gb * lz;
        Z[i] = -gb * le + g * lz;
    }
    o.shat = x1 * x2 * s_lab;
    o.x1 = x1;
    o.x2 = x2;
    o.logtau = log(x1 * x2);
    o.jac = jac;
}

// Invariant store in private registers (the weight entry point).
// Rows of the per-event invariant store: one per distinct invariant, plus
// row kMaxUniq holding 1.0 (the pad of the channel products).
constexpr int kQRows = kMaxUniq + 1;
struct RegQ {
    double v[kQRows];
    __device__ __forceinline__ void set(int u, double x) { v[u] = x; }
    __device__ __forceinline__ double get(int u) const { return v[u]; }
};

// ---------------------------------------------------------------------------
// Integrand and local channel weight, from momenta supplied by an accessor
// get(k, c) for final-state particle k (0-based) and component c, plus p_a.
// ---------------------------------------------------------------------------
// Loops over final-state particles run over a compile-time bound NF with a
// wave-uniform guard, so get(k, c) is always called with a constant k (the
// momenta stay in statically indexed registers).
template <int NF, class Get>
__device__ __forceinline__ double inv_q2(const ProcessTab* __restrict__ pt, int u, double pae, double pax, double pay,
                                         double paz, Get get) {
    double qe = 0.0, qx = 0.0, qy = 0.0, qz = 0.0;
    const uint32_t set = pt->uq[u].set;
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        if (set & (1u << k)) {
            qe += get(k, 0);
            qx += get(k, 1);
            qy += get(k, 2);
            qz += get(k, 3);
        }
    }
    if (pt->uq[u].t) {
        qe = pae - qe;
        qx = pax - qx;
        qy = pay - qy;
        qz = paz - qz;
    }
    return qe * qe - qx * qx - qy * qy - qz * qz;
}

// Returns alpha * f; *alpha_out receives alpha.  `logtau` = log(x1 x2).
// NF bounds the number of final-state particles of the process.  q is the
// per-event store of the invariants' channel-weight denominators, indexed by
// invariant (q.set(u, v), q.get(u)): an LDS column in the sampling kernels.
template <bool MIX, int NF, class Get, class Q>
__device__ __forceinline__ double integrand_alpha(const ProcessTab* __restrict__ pt, int chan_in_proc, double x1,
                                                  double x2, double logtau, double pae, double pax, double pay,
                                                  double paz, Get get, Q& q, double& alpha_out) {
    double f = 1.0;
    const int n = pt->n_final;
    if (pt->pdf) {
        // x1^a x2^a = tau^a; integer b by multiplication
        double u1 = 1.0 - x1, u2 = 1.0 - x2;
        double b1, b2;
        if (pt->pdf_b_int > 0) {
            b1 = ipow_any(u1, pt->pdf_b_int);
            b2 = ipow_any(u2, pt->pdf_b_int);
        } else {
            b1 = t_pow<MIX>(u1, pt->pdf_b);
            b2 = t_pow<MIX>(u2, pt->pdf_b);
        }
        f = t_exp<MIX>(pt->pdf_a * logtau) * b1 * b2;
    }
    if (pt->pt_min2 > 0.0) {
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            if (i < n) {
                double px = get(i, 1), py = get(i, 2);
                if (!(px * px + py * py > pt->pt_min2)) f = 0.0;
            }
        }
    }
    if (pt->ang >= 0) {
#pragma unroll
        for (int i = 0; i < NF; ++i) {
            if (i == pt->ang) {
                double px = get(i, 1), py = get(i, 2), pz = get(i, 3);
                double c = pz / sqrt(px * px + py * py + pz * pz);
                f *= 1.0 + c * c;
            }
        }
    }
    // each distinct invariant once: its integrand factor (product of the
    // denominators, one reciprocal) and its channel-weight denominator
    const int nu = pt->n_uniq;
    const int nc = pt->n_chan;
    double fden = 1.0;
    for (int u = 0; u < nu; ++u) {
        const UniqSpec& us = pt->uq[u];
        const double q2 = inv_q2<NF>(pt, u, pae, pax, pay, paz, get);
        if (us.fkind == 1) {
            const double d = q2 - us.fa;
            fden *= d * d + us.fb;
        } else if (us.fkind == 2) {
            fden *= fabs(q2) + us.fa;
        }
        if (nc > 1) {
            double dd;
            if (us.massive > 0) {
                const double d = q2 - us.am2;
                dd = d * d + us.amw2;
            } else {
                const double d = fabs(q2) + pt->alpha_mu2;
                dd = d * d;
            }
            q.set(u, dd);
        }
    }
    if (pt->n_fprop > 0) f /= fden;
    double alpha = 1.0;
    if (nc > 1 && ((pt->chan_prior >> chan_in_proc) & 1)) {
        alpha = pt->prior_share;
    } else if (nc > 1) {
        q.set(kMaxUniq, 1.0);
        double den = 0.0, mine = 0.0;
        const uint32_t prior = pt->chan_prior;
        for (int c = 0; c < nc; ++c) {
            if ((prior >> c) & 1) continue;
            // product over the channel's invariants in ascending order, four
            // independent loads per round (short rounds padded with the 1.0 row)
            double D = 1.0;
            uint32_t m = pt->chan_mask[c];
            while (m) {
                int u[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    u[j] = m ? __builtin_ctz(m) : kMaxUniq;
                    m &= m - 1;
                }
                const double v0 = q.get(u[0]), v1 = q.get(u[1]), v2 = q.get(u[2]), v3 = q.get(u[3]);
                D = D * v0 * v1 * v2 * v3;
            }
            const double P = 1.0 / D;
            den += P;
            if (c == chan_in_proc) mine = P;
        }
        alpha = pt->tree_share * (mine / den);
    }
    alpha_out = alpha;
    return alpha * f;
}

}  // namespace msx

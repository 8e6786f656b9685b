// sl_device.hpp -- device building blocks of the spin-lattice step on gfx950.
//
// Everything here is __host__ __device__ so that the integer logic (site
// numbering, division by run-time constants, Philox) can also be checked on
// the CPU.  Floating-point formulas are written once, templated on the
// storage precision T (float or double).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sl {

// ------------------------------------------------------------- constants
// CODATA 2018 in metal units (Angstrom, ps, eV, amu, K, T).
constexpr double kKB = 8.617333262e-5;        // eV/K
constexpr double kHBAR = 6.582119569e-4;      // eV ps
constexpr double kMUB = 5.7883818060e-5;      // eV/T
constexpr double kGAMMA = 2.0 * kMUB / kHBAR; // rad/(ps T), g = 2
// amu (A/ps)^2 -> eV
constexpr double kMVV2E = 1.66053906660e-27 * 1.0e4 / 1.602176634e-19;
// fixed-point scale of the per-cell electron-phonon energy accumulators
constexpr double kFIX = 4503599627370496.0;   // 2^52 units per eV
constexpr double kTWO_M32 = 2.3283064365386963e-10;  // 2^-32

// ------------------------------------------------------- division helper
// Quotient of n < 2^31 by a fixed divisor d >= 1 with one high multiply
// (Granlund-Montgomery "division by invariant integers"):
//   l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1,
//   q = (mulhi(n, m) + n) >> l.
struct FastDiv {
    uint32_t d, m, l;
};

__host__ __device__ inline FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.l = l;
    f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1ull);
    return f;
}

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, b);
#else
    return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f)
{
    return (mulhi32(n, f.m) + n) >> f.l;
}

// ---------------------------------------------------------------- Philox
// Philox4x32-10 (Salmon et al., SC'11) from its definition: per round two
// 32x32 -> 64-bit products of counter words 0 and 2 with the round
// multipliers, the high halves mixed with the other words and the key, the
// key advanced by the Weyl increments between rounds.
struct U4 {
    uint32_t x, y, z, w;
};

__host__ __device__ inline U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32 -> 64-bit product per multiplier (v_mad_u64_u32 on gfx950)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Three standard normals from one Philox block keyed by (seed, run) at
// counter (site id, step low, step high, stream): words -> open-interval
// uniforms (w + 1/2) 2^-32 -> two Box-Muller pairs, the fourth normal
// dropped.  The single-precision variant keeps the top 24 bits of each word
// ((w >> 8) + 1/2) 2^-24, which a float holds exactly.
template <typename T> struct Normals3 {
    T a, b, c;
};

__device__ inline Normals3<double> normals3_f64(uint32_t seed, uint32_t run, uint32_t id,
                                                int64_t step, uint32_t stream)
{
    U4 ctr{id, (uint32_t)((uint64_t)step & 0xFFFFFFFFu), (uint32_t)((uint64_t)step >> 32),
           stream};
    U4 w = philox4x32_10(ctr, seed, run);
    double u0 = ((double)w.x + 0.5) * kTWO_M32;
    double u1 = ((double)w.y + 0.5) * kTWO_M32;
    double u2 = ((double)w.z + 0.5) * kTWO_M32;
    double u3 = ((double)w.w + 0.5) * kTWO_M32;
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    double s1, c1, c3;
    sincospi(2.0 * u1, &s1, &c1);
    c3 = cospi(2.0 * u3);
    return {r0 * c1, r0 * s1, r1 * c3};
}

__device__ inline Normals3<float> normals3_f32(uint32_t seed, uint32_t run, uint32_t id,
                                               int64_t step, uint32_t stream)
{
    U4 ctr{id, (uint32_t)((uint64_t)step & 0xFFFFFFFFu), (uint32_t)((uint64_t)step >> 32),
           stream};
    U4 w = philox4x32_10(ctr, seed, run);
    float u0 = ((float)(w.x >> 8) + 0.5f) * 5.9604644775390625e-8f;   // 24-bit uniforms
    float u1 = ((float)(w.y >> 8) + 0.5f) * 5.9604644775390625e-8f;
    float u2 = ((float)(w.z >> 8) + 0.5f) * 5.9604644775390625e-8f;
    float u3 = ((float)(w.w >> 8) + 0.5f) * 5.9604644775390625e-8f;
    // hardware log2 / sqrt / sin / cos (a few ulp): the single-precision
    // path is compared with double precision statistically, not per
    // trajectory.  -2 ln u = -2 ln(2) log2(u); u >= 2^-25 is never denormal.
    float r0 = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u0));
    float r1 = __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u2));
    float s1, c1;
    __sincosf(6.28318530717958648f * u1, &s1, &c1);
    float c3 = __cosf(6.28318530717958648f * u3);
    return {r0 * c1, r0 * s1, r1 * c3};
}

template <typename T> __device__ inline Normals3<T> normals3(uint32_t, uint32_t, uint32_t,
                                                             int64_t, uint32_t);
template <> __device__ inline Normals3<double> normals3<double>(uint32_t s, uint32_t r,
                                                                uint32_t i, int64_t st,
                                                                uint32_t sm)
{
    return normals3_f64(s, r, i, st, sm);
}
template <> __device__ inline Normals3<float> normals3<float>(uint32_t s, uint32_t r,
                                                              uint32_t i, int64_t st,
                                                              uint32_t sm)
{
    return normals3_f32(s, r, i, st, sm);
}

// ------------------------------------------------------ exact LLG flow
// Constant precession vector w over a time tau (Eq. (1), Landau-Lifshitz
// form).  With e = w/|w|, u = s.e, phi = |w| tau/(1+alpha^2) and
// E = exp(-alpha phi), tan(theta/2) shrinks by E while the transverse part
// turns right-handedly about e by phi.  Using
//   cos(theta') = ((1+u) - (1-u) E^2) / D,  sin(theta') = 2 E |s_perp| / D,
//   D = (1+u) + (1-u) E^2,
// the new spin is cos(theta') e + (2E/D) R_phi(s_perp) with no division by
// |s_perp| (finite for s along +e or -e).  Renormalised in double.
// For a unit input the squared length before the renormalisation is 1 up to
// rounding; an input that is not finite, or whose length is off by more than
// a few 1e-5, moves it by more than kNormTol and sets `bad` (the run's
// numeric watchdog).
template <typename T> struct V3 {
    T x, y, z;
};

constexpr double kNormTol = 1.0e-4;

__device__ inline void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ inline void sin_cos(float x, float* s, float* c) { __sincosf(x, s, c); }
__device__ inline double expo(double x) { return exp(x); }
__device__ inline float expo(float x) { return __expf(x); }

template <typename T>
__device__ inline V3<T> llg_flow(V3<T> s, V3<T> w, T alpha, T tau, T inv1pa2, bool& bad)
{
    T wn2 = w.x * w.x + w.y * w.y + w.z * w.z;
    if (!(wn2 > T(0))) {
        bad |= !(s.x * s.x + s.y * s.y + s.z * s.z < T(2));
        return s;
    }
    T wn = sqrt(wn2);
    T iw = T(1) / wn;
    V3<T> e{w.x * iw, w.y * iw, w.z * iw};
    T u = s.x * e.x + s.y * e.y + s.z * e.z;
    V3<T> p{s.x - u * e.x, s.y - u * e.y, s.z - u * e.z};
    T phi = wn * tau * inv1pa2;
    T E = expo(-alpha * phi);
    T E2 = E * E;
    T D = (T(1) + u) + (T(1) - u) * E2;
    T iD = T(1) / D;
    T ct = ((T(1) + u) - (T(1) - u) * E2) * iD;
    T f = T(2) * E * iD;
    T sn, cs;
    sin_cos(phi, &sn, &cs);
    V3<T> ex{e.y * p.z - e.z * p.y, e.z * p.x - e.x * p.z, e.x * p.y - e.y * p.x};
    double ox = (double)(ct * e.x + f * (cs * p.x + sn * ex.x));
    double oy = (double)(ct * e.y + f * (cs * p.y + sn * ex.y));
    double oz = (double)(ct * e.z + f * (cs * p.z + sn * ex.z));
    const double n2 = ox * ox + oy * oy + oz * oz;
    bad |= !(fabs(n2 - 1.0) < kNormTol);
    double inv = 1.0 / sqrt(n2);
    return {(T)(ox * inv), (T)(oy * inv), (T)(oz * inv)};
}

// Single precision: the same flow with the hardware reciprocal, reciprocal
// square root, exponential and sine/cosine (about 1 ulp each).  The result
// is renormalised in double: its squared norm is 1 + eps with |eps| of a
// few float ulps, so 1/sqrt(1 + eps) = 1 - eps/2 + 3 eps^2/8 to within
// 5|eps|^3/16 (below 1e-15 for |eps| < 1e-5); larger eps takes the exact
// reciprocal square root.
__device__ inline V3<float> llg_flow(V3<float> s, V3<float> w, float alpha, float tau,
                                     float inv1pa2, bool& bad)
{
    const float wn2 = w.x * w.x + w.y * w.y + w.z * w.z;
    if (!(wn2 > 0.0f)) {
        bad |= !(s.x * s.x + s.y * s.y + s.z * s.z < 2.0f);
        return s;
    }
    const float iw = __builtin_amdgcn_rsqf(wn2);
    const float wn = wn2 * iw;
    const V3<float> e{w.x * iw, w.y * iw, w.z * iw};
    const float u = s.x * e.x + s.y * e.y + s.z * e.z;
    const V3<float> p{s.x - u * e.x, s.y - u * e.y, s.z - u * e.z};
    const float phi = wn * tau * inv1pa2;
    const float E = __expf(-alpha * phi);
    const float E2 = E * E;
    const float D = (1.0f + u) + (1.0f - u) * E2;
    const float iD = __builtin_amdgcn_rcpf(D);
    const float ct = ((1.0f + u) - (1.0f - u) * E2) * iD;
    const float f = 2.0f * E * iD;
    float sn, cs;
    __sincosf(phi, &sn, &cs);
    const V3<float> ex{e.y * p.z - e.z * p.y, e.z * p.x - e.x * p.z, e.x * p.y - e.y * p.x};
    const double ox = (double)(ct * e.x + f * (cs * p.x + sn * ex.x));
    const double oy = (double)(ct * e.y + f * (cs * p.y + sn * ex.y));
    const double oz = (double)(ct * e.z + f * (cs * p.z + sn * ex.z));
    const double eps = (ox * ox + oy * oy + oz * oz) - 1.0;
    bad |= !(fabs(eps) < kNormTol);
    const double inv = fabs(eps) < 1.0e-5 ? 1.0 + eps * (-0.5 + 0.375 * eps)
                                          : 1.0 / sqrt(1.0 + eps);
    return {(float)(ox * inv), (float)(oy * inv), (float)(oz * inv)};
}

// ------------------------------------------------------------- lattice
// Site numbering.  Colour k of a site is (x+y+z) mod 2 on the simple-cubic
// lattice, 2b + (x+y+z) mod 2 on bcc (b = 0 corner, 1 body centre), and the
// basis site b itself on fcc (b = 0 corner, 1..3 the face centres of the xy,
// xz and yz faces: no two nearest neighbours share a sublattice).  Inside the
// device arrays the sites of one colour are contiguous, in rows along x:
//   sc, bcc (checkerboard, par = 1): internal = k H + xh + (Lx/2)(y + Ly z),
//     x = 2 xh + ((k + y + z) & 1), H = Lx Ly Lz / 2;
//   fcc (par = 0): internal = k H + x + Lx (y + Ly z), H = Lx Ly Lz,
// so one colour pass streams one contiguous block.  `Lxh` is the length of a
// row of one colour (Lx / 2 or Lx).  The canonical (public) number is
// ((z Ly + y) Lx + x) nb + b.
struct Geom {
    int32_t Lx, Ly, Lz;   // unit cells per dimension (even for the checkerboard)
    int32_t Lxh;          // sites of one colour per row: Lx / 2 (par) or Lx
    int32_t H;            // sites per colour
    int32_t nb;           // basis atoms per cell (1 sc, 2 bcc, 4 fcc)
    int32_t C;            // colours (2 sc, 4 bcc, 4 fcc)
    int32_t par;          // 1: checkerboard rows of half length; 0: full rows
    FastDiv divH, divLxh, divLy;
};

struct Site {
    int32_t x, y, z, b, k;
};

// Axes along which basis site b is shifted by half a lattice constant from
// the cell corner (bit 0 x, bit 1 y, bit 2 z): bcc body centre all three;
// fcc face centres (xy), (xz), (yz).
__host__ __device__ inline uint32_t basis_half_bits(int32_t nb, int32_t b)
{
    if (nb == 2) return b ? 7u : 0u;
    if (nb == 4) return b == 0 ? 0u : (b == 1 ? 3u : (b == 2 ? 5u : 6u));
    return 0u;
}

__host__ __device__ inline Site decode_site(const Geom& g, uint32_t idx)
{
    Site s;
    uint32_t k = fdiv(idx, g.divH);
    uint32_t l = idx - k * (uint32_t)g.H;
    uint32_t r = fdiv(l, g.divLxh);
    uint32_t xh = l - r * (uint32_t)g.Lxh;
    uint32_t z = fdiv(r, g.divLy);
    uint32_t y = r - z * (uint32_t)g.Ly;
    s.k = (int32_t)k;
    s.b = g.nb == 2 ? (int32_t)(k >> 1) : (g.nb == 4 ? (int32_t)k : 0);
    s.y = (int32_t)y;
    s.z = (int32_t)z;
    s.x = g.par ? 2 * (int32_t)xh + (int32_t)((k + y + z) & 1u) : (int32_t)xh;
    return s;
}

// internal index of the site at cell (x, y, z) (already wrapped) and basis b
__host__ __device__ inline int32_t encode_site(const Geom& g, int32_t x, int32_t y, int32_t z,
                                               int32_t b)
{
    if (!g.par) return b * g.H + x + g.Lxh * (y + g.Ly * z);
    int32_t par = (x + y + z) & 1;
    int32_t k = (g.nb == 2) ? (2 * b + par) : par;
    return k * g.H + (x >> 1) + g.Lxh * (y + g.Ly * z);
}

__host__ __device__ inline int32_t canonical_of(const Geom& g, const Site& s)
{
    return ((s.z * g.Ly + s.y) * g.Lx + s.x) * g.nb + s.b;
}

__host__ __device__ inline int32_t wrapi(int32_t v, int32_t L)
{
    return v < 0 ? v + L : (v >= L ? v - L : v);
}

// -------------------------------------------------------- launch tables
// A single run's launch tables are arithmetic: entry q of a table is (run,
// q * tile), or, ordered for the XCDs (block b runs on XCD b mod 8), the
// entries of the m tiles dealt so that XCD x receives the contiguous range
// x * per .. x * per + per - 1 (per = ceil(m / 8)) in order: with a = the
// number of full ranges and r the length of the partial one, output q takes
// tile x * per + j where (j, x) enumerates j = 0, 1, ... with x over the
// ranges still holding a tile at j.  Tables shorter than 16 keep their order.
constexpr int kXcdCount = 8;

struct TableFill {
    int32_t off[6], m[6], tile[6], xcd[6];   // six int2 tables, offsets in entries
    int32_t n_int2;                           // entries of the six tables together
    int32_t slot;                             // the run
    int32_t rl_n, pl_n;                       // run list and persistent list (0 or 1 each)
};

__host__ __device__ inline int2 fill_entry(const TableFill& f, int k, int32_t q, int32_t slot)
{
    const int32_t m = f.m[k];
    int32_t src = q;
    if (f.xcd[k] && m >= 2 * kXcdCount) {
        const int32_t per = (m + kXcdCount - 1) / kXcdCount;
        const int32_t a = m / per, r = m - a * per;
        int32_t j, x;
        if (q < r * (a + 1)) {
            j = q / (a + 1);
            x = q - j * (a + 1);
        } else {
            const int32_t q2 = q - r * (a + 1);
            j = r + q2 / a;
            x = q2 - (q2 / a) * a;
        }
        src = x * per + j;
    }
    return make_int2(slot, src * f.tile[k]);
}

}  // namespace sl

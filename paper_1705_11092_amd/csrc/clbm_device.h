// clbm_device.h -- device-side pieces of the D2Q9 cascaded LBM step for gfx950.
//
// The per-node collision of Fei & Luo (Eq. 12 with Eqs. 8, 14, 15, then the
// back-transform of Eq. 9) is evaluated here in closed form: the products
// with M, N(u), N^-1(u) and M^-1 are expanded by hand into sums over the
// populations, and everything is carried as deviations from the rest state
// (f_i - w_i rho0, rho - rho0, moments minus their equilibrium values) so
// that FP32 keeps its digits for the small departures that matter.
//
// Notation: g_i = f_i - w_i rho0 (stored), dr = rho - rho0, j = sum f e,
// u = (j + F/2)/rho (Eq. 15).  Raw moments of g:
//   kxx = sum g ex^2, kyy = sum g ey^2, kxy = sum g ex ey,
//   kxxy = sum g ex^2 ey, kxyy = sum g ex ey^2, kxxyy = sum g ex^2 ey^2.
// The rest state contributes rho0/3 to k20 and k02 and rho0/9 to k22 and
// nothing else.  Central moments k~mn (Eq. 2) follow from the binomial
// shift of the raw ones, with j = rho u - F/2 substituted, which gives the
// equilibrium-deviation forms used below:
//   k~20 - rho/3 = kxx - dr/3 - rho ux^2 + ux Fx
//   k~11         = kxy - rho ux uy + (ux Fy + uy Fx)/2
//   k~21         = kxxy - 2 ux kxy - uy (kxx + rho0/3) + 2 rho ux^2 uy
//                  - ux^2 Fy/2 - ux uy Fx
//   k~22 - rho/9 = kxxyy - dr/9 - 2 ux kxyy - 2 uy kxxy + ux^2 kyy + uy^2 kxx
//                  + (ux^2 + uy^2) rho0/3 + 4 ux uy kxy - 3 rho ux^2 uy^2
//                  + ux uy (uy Fx + ux Fy)
// and symmetric ones with x and y exchanged.  The collision then changes
// each central moment by Delta T~ = T~* - T~ (Eq. 12: -s (T~ - T~eq) plus the
// force term, and exactly F in the first-order slots), and only that change
// is carried back through N^-1(u) (the inverse binomial shift) and M^-1
// (Appendix): g* = g + M^-1 N^-1 Delta T~.  Carrying the small change rather
// than the whole post-collision state keeps FP32 rounding unbiased: the
// population values are rounded once, in the final add, while the force
// increment enters as F itself instead of as F added to rho u (whose FP32
// rounding has the same sign at every node and step, a steady drift).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace clbm {

// Eq. (1) order.
__host__ __device__ constexpr int ex_of(int i) { return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0; }
__host__ __device__ constexpr int ey_of(int i) { return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0; }
__host__ __device__ constexpr int opp_of(int i) { return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5); }
static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(3) == 1 && opp_of(4) == 2, "opp");
static_assert(opp_of(5) == 7 && opp_of(6) == 8 && opp_of(7) == 5 && opp_of(8) == 6, "opp");

// Rest weights w_i = f_i^eq(rho = 1, u = 0).
template <typename R>
__host__ __device__ __forceinline__ R weight(int i)
{
    return i == 0 ? R(4) / R(9) : (i <= 4 ? R(1) / R(9) : R(1) / R(36));
}

// ---- storage conversions ---------------------------------------------------

enum StorageKind { ST_F64 = 0, ST_F32 = 1, ST_F16 = 2, ST_BF16 = 3, ST_F16_SR = 4, ST_BF16_SR = 5 };

template <int ST> struct Storage;

template <> struct Storage<ST_F64> {
    using T = double;  // stored element
    using R = double;  // arithmetic
    static constexpr bool kDither = false;
    static __device__ __forceinline__ R to_r(T v) { return v; }
    static __device__ __forceinline__ T from_r(R v) { return v; }
};

template <> struct Storage<ST_F32> {
    using T = float;
    using R = float;
    static constexpr bool kDither = false;
    static __device__ __forceinline__ R to_r(T v) { return v; }
    static __device__ __forceinline__ T from_r(R v) { return v; }
};

// The FP32 value v as computed, opaque to the optimiser.  gfx950 can fuse a
// multiply-add and the conversion of its result to binary16 into one
// instruction (v_fma_mixlo_f16) that rounds once, to 16 bits, instead of
// twice; the compiler does so in some kernels and not in others, which would
// then store different bits for the same node update.  Passing the FP32
// result through an empty asm statement keeps the conversion a separate
// instruction everywhere, at no cost in instructions.
__device__ __forceinline__ float fp32_value(float v)
{
    asm("" : "+v"(v));
    return v;
}

template <> struct Storage<ST_F16> {
    using T = _Float16;
    using R = float;
    static constexpr bool kDither = false;
    static __device__ __forceinline__ R to_r(T v) { return (float)v; }
    static __device__ __forceinline__ T from_r(R v) { return (_Float16)fp32_value(v); }  // RNE
};

// bfloat16: gfx950 converts FP32 to bfloat16 in hardware, rounding to
// nearest even (v_cvt_pk_bf16_f32).
template <> struct Storage<ST_BF16> {
    using T = __bf16;
    using R = float;
    static constexpr bool kDither = false;
    static __device__ __forceinline__ R to_r(T v) { return (float)v; }
    static __device__ __forceinline__ T from_r(R v) { return (__bf16)fp32_value(v); }
};

// Stochastically rounded 16-bit storage.  A value that changes by a few
// units in the last place per step (a slowly evolving flow, a small body
// force) is rounded the same way step after step by round-to-nearest, a
// drift that accumulates.  Here each stored value v becomes its lower or
// upper 16-bit neighbour with probabilities that make it exact on average:
// gfx950's stochastic-rounding conversions (v_cvt_sr_f16_f32,
// v_cvt_sr_bf16_f32) round up when the discarded fraction of v plus a
// uniform random fraction, taken from the high bits of a 32-bit operand,
// reaches one ulp (measured on MI355X: P(up) equals the fraction for both
// types, signs round by magnitude, binary16 subnormals are unbiased).  The
// operand comes from a hash of the node index and the node's own FP32
// values, so it is deterministic (a lattice gives the same bits alone or in
// any batch, in any launch shape) and changes from step to step with the
// state.
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bfloat2_t __attribute__((ext_vector_type(2)));

template <> struct Storage<ST_F16_SR> {
    using T = _Float16;
    using R = float;
    static constexpr bool kDither = true;
    static __device__ __forceinline__ R to_r(T v) { return (float)v; }
    static __device__ __forceinline__ T from_r(R v) { return (_Float16)fp32_value(v); }
    static __device__ __forceinline__ T from_r_sr(R v, uint32_t rnd)
    {
        return __builtin_amdgcn_cvt_sr_f16_f32(half2_t{}, v, rnd, false)[0];
    }
    // Two values into the low and high halves of one register.
    static __device__ __forceinline__ half2_t from_r_sr2(R a, uint32_t ra, R b, uint32_t rb)
    {
        return __builtin_amdgcn_cvt_sr_f16_f32(
            __builtin_amdgcn_cvt_sr_f16_f32(half2_t{}, a, ra, false), b, rb, true);
    }
};

template <> struct Storage<ST_BF16_SR> {
    using T = __bf16;
    using R = float;
    static constexpr bool kDither = true;
    static __device__ __forceinline__ R to_r(T v) { return (float)v; }
    static __device__ __forceinline__ T from_r(R v) { return (__bf16)fp32_value(v); }
    static __device__ __forceinline__ T from_r_sr(R v, uint32_t rnd)
    {
        return __builtin_amdgcn_cvt_sr_bf16_f32(bfloat2_t{}, v, rnd, false)[0];
    }
    static __device__ __forceinline__ bfloat2_t from_r_sr2(R a, uint32_t ra, R b, uint32_t rb)
    {
        return __builtin_amdgcn_cvt_sr_bf16_f32(
            __builtin_amdgcn_cvt_sr_bf16_f32(bfloat2_t{}, a, ra, false), b, rb, true);
    }
};

// Two values rounded to nearest into the storage type.  For the 16-bit
// types one packed conversion (v_cvt_pk_f16_f32, v_cvt_pk_bf16_f32) rounds
// both, with the same round-to-nearest-even as the conversion of one value,
// so a value gets the same bits whether it is converted alone or in a pair.
// dst points to two consecutive elements (the pair lands as one 32-bit
// word for the 16-bit types).
typedef float float2v_t __attribute__((ext_vector_type(2)));
template <int ST>
__device__ __forceinline__ void round_pair(typename Storage<ST>::R a, typename Storage<ST>::R b,
                                           typename Storage<ST>::T *dst)
{
    using S = Storage<ST>;
    if constexpr (ST == ST_F16) {
        const half2_t h = __builtin_convertvector(float2v_t{fp32_value(a), fp32_value(b)}, half2_t);
        __builtin_memcpy(dst, &h, sizeof h);
    } else if constexpr (ST == ST_BF16) {
        const bfloat2_t h = __builtin_convertvector(float2v_t{fp32_value(a), fp32_value(b)}, bfloat2_t);
        __builtin_memcpy(dst, &h, sizeof h);
    } else {
        dst[0] = S::from_r(a);
        dst[1] = S::from_r(b);
    }
}

// 32-bit integer finaliser: xor-shift-multiply in MurmurHash3's fmix32
// structure, with the shifts and multipliers of "lowbias32", found by
// Chris Wellons' hash-prospector search (public domain, 2018).
__device__ __forceinline__ uint32_t hash32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return h;
}

// Random operand of population i of a node with hash h: a Weyl step of
// the golden-ratio increment, so each direction's operand is uniform
// (h is) and the nine of a node spread evenly over [0, 2^32).  One add per
// value, where a multiply would cost four.
__device__ __forceinline__ uint32_t sr_operand(uint32_t h, int i)
{
    return h + (uint32_t)i * 0x9e3779b9u;
}

// ---- relaxation parameters in the arithmetic type --------------------------

enum SchemeKind { SCH_CONSISTENT = 0, SCH_GUO_LBL = 1 };

template <typename R>
struct Rates {
    R nap, nam;       // -(sb + s2)/2, -(sb - s2)/2: k~20, k~02 relax as a trace
                      // at sb and a deviator at s2 (Eq. 12)
    R ns2, ns3, ns4;  // -s2, -s3, -s4
    R h3t;            // (1 - s3/2) cs^2: third-order force weight of Eq. (12);
                      // 0 for the scheme of Sec. III A, whose force moments
                      // (Eq. 19) stop at first order
    R g1;             // s1/2 + 1 - s2/2: first-order change per unit force (Eq. 21)
    R h2;             // 1 - s2/2 (force weight of Eq. 21)
    R rho0, r3;       // rho0 and rho0/3
};

// ---- the node update -------------------------------------------------------

// 1/rho.  In FP32 on the GPU the hardware reciprocal (1 ulp) replaces the
// correctly rounded division, which costs about ten instructions; FP64 keeps
// the exact division.
__host__ __device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__host__ __device__ __forceinline__ float recip(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

// Back-transform (Eq. 9): from the post-collision central moments, given as
// deviations, to post-collision deviations g*.
//   mx, my   : rho ux and rho uy, passed exactly (j + F/2), so that the
//              rebuilt first moments are c10 + mx to one rounding and
//              momentum is conserved without a drift from rho * (mx / rho)
//   c10, c01 : k~10*, k~01*
//   p, q     : k~20* - rho/3 and k~02* - rho/3
//   a5..a8   : k~11*, k~21*, k~12*, k~22* - rho/9
template <typename R>
__host__ __device__ __forceinline__ void from_central(R dr, R rho, R mx, R my, R ux, R uy, R c10, R c01,
                                                      R p, R q, R a5, R a6, R a7, R a8, R g[9])
{
    const R third = R(1) / R(3);
    const R ninth = R(1) / R(9);
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    const R c20 = rho * third + p;  // full k~20*
    const R c02 = rho * third + q;  // full k~02*
    // Raw moments (inverse binomial shift) minus the rest-state raw moments;
    // rho u^a u^b is written (rho ux) ux... from the exact momentum.
    const R r10 = c10 + mx;
    const R r01 = c01 + my;
    const R r20 = dr * third + p + R(2) * ux * c10 + mx * ux;
    const R r02 = dr * third + q + R(2) * uy * c01 + my * uy;
    const R r11 = a5 + ux * c01 + uy * c10 + mx * uy;
    const R r21 = a6 + R(2) * ux * a5 + uy * c20 + uxx * c01 + R(2) * uxy * c10 + mx * uxy;
    const R r12 = a7 + R(2) * uy * a5 + ux * c02 + uyy * c10 + R(2) * uxy * c01 + my * uxy;
    const R r22 = dr * ninth + a8 + R(2) * ux * a7 + R(2) * uy * a6 + uxx * c02 + uyy * c20 +
                  R(4) * uxy * a5 + R(2) * ux * uyy * c10 + R(2) * uxx * uy * c01 + mx * ux * uyy;
    // M^-1 (Appendix), row by row.
    const R h = R(0.5), qr = R(0.25);
    g[0] = dr - (r20 + r02) + r22;
    g[1] = h * (r10 + r20 - r12 - r22);
    g[2] = h * (r01 + r02 - r21 - r22);
    g[3] = h * (-r10 + r20 + r12 - r22);
    g[4] = h * (-r01 + r02 + r21 - r22);
    g[5] = qr * (r11 + r21 + r12 + r22);
    g[6] = qr * (-r11 + r21 - r12 + r22);
    g[7] = qr * (r11 - r21 - r12 + r22);
    g[8] = qr * (-r11 - r21 + r12 + r22);
}

// g += M^-1 N^-1(u) D for a change D of the central moments about u
// (Eq. 9 applied to the change, D0 = 0):
//   d10, d01 : D k~10, D k~01
//   d20, d02 : D k~20, D k~02
//   d11..d22 : D k~11, D k~21, D k~12, D k~22
// N^-1(u) is the binomial shift of the moments by u; it factorises into a
// shift along x (k_mn -> k_mn + m ux k_(m-1)n + ...) followed by one along
// y, which is how it is applied here (14 multiply-adds instead of the 28 of
// the expanded rows).  M^-1 (Appendix) is then taken on sums and
// differences of the raw moments, each population's half or quarter folded
// into its update.
template <typename R>
__host__ __device__ __forceinline__ void add_back(R g[9], R ux, R uy, R d10, R d01, R d20, R d02, R d11,
                                                  R d21, R d12, R d22)
{
    const R ux2 = ux + ux, uy2 = uy + uy, uxx = ux * ux, uyy = uy * uy;
    // Shift along x (the moments of order 0 in x are unchanged).
    const R t20 = d20 + ux2 * d10;
    const R t11 = d11 + ux * d01;
    const R t21 = d21 + ux2 * d11 + uxx * d01;
    const R t12 = d12 + ux * d02;
    const R t22 = d22 + ux2 * d12 + uxx * d02;
    // Shift along y: the raw moments r_mn (r10 = d10, r01 = d01, r20 = t20).
    const R r02 = d02 + uy2 * d01;
    const R r11 = t11 + uy * d10;
    const R r21 = t21 + uy * t20;
    const R r12 = t12 + uy2 * t11 + uyy * d10;
    const R r22 = t22 + uy2 * t21 + uyy * t20;
    // M^-1, row by row.
    const R h = R(0.5), qr = R(0.25);
    const R a = t20 - r22, b = d10 - r12;
    const R c = r02 - r22, e = d01 - r21;
    const R p = r22 + r11, q = r22 - r11, m = r21 + r12, n = r21 - r12;
    g[0] = g[0] + (r22 - (t20 + r02));
    g[1] = g[1] + h * (a + b);
    g[3] = g[3] + h * (a - b);
    g[2] = g[2] + h * (c + e);
    g[4] = g[4] + h * (c - e);
    g[5] = g[5] + qr * (p + m);
    g[7] = g[7] + qr * (p - m);
    g[6] = g[6] + qr * (q + n);
    g[8] = g[8] + qr * (q - n);
}

// One collision in place: g holds pre-collision deviations on entry and
// post-collision deviations on exit.  F is the force density at the node.
template <typename R, int SCH>
__host__ __device__ __forceinline__ void collide(R g[9], R Fx, R Fy, const Rates<R> &rt)
{
    const R third = R(1) / R(3);
    const R ninth = R(1) / R(9);
    const R h = R(0.5);

    // Eq. (11) on deviations, and the raw moments of g (Eq. 2).  (Regrouping
    // these sums so that jx shares kxyy's rounding, or dr kxx's, saves a few
    // adds but made the FP32 drift of slow steady flows several times worse:
    // a 124^2 Kolmogorov flow at tau 1.36 went from 3e-6 to 1.4e-5 relative
    // after 40,000 steps in a host emulation of the kernel.)
    const R sx = g[1] + g[3];
    const R sy = g[2] + g[4];
    const R kxxyy = (g[5] + g[6]) + (g[7] + g[8]);
    const R dr = g[0] + sx + sy + kxxyy;
    const R jx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const R jy = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    const R kxx = sx + kxxyy;
    const R kyy = sy + kxxyy;
    const R kxy = (g[5] + g[7]) - (g[6] + g[8]);
    const R kxxy = (g[5] + g[6]) - (g[7] + g[8]);
    const R kxyy = (g[5] + g[8]) - (g[6] + g[7]);
    const R rho = rt.rho0 + dr;
    const R inv = recip(rho);
    const R hFx = h * Fx, hFy = h * Fy;
    const R mx = jx + hFx;  // rho ux (Eq. 15)
    const R my = jy + hFy;
    const R ux = mx * inv;
    const R uy = my * inv;
    const R uxx = ux * ux, uyy = uy * uy, uxy = ux * uy;
    const R ux2 = ux + ux, uy2 = uy + uy;

    // Central moments (Eq. 6) as deviations from T~eq (Eq. 8).  With
    // j = rho u - F/2 the shift of the raw moments simplifies to
    //   k~11         = kxy - uy jx + ux Fy/2
    //   k~20 - rho/3 = kxx - dr/3 - ux (jx - Fx/2)
    //   k~21         = kxxy - uy (kxx + rho0/3) - 2 ux k~11 + ux^2 Fy/2
    //   k~22 - rho/9 = kxxyy - dr/9 - 2 uy k~21 - 2 ux k~12 - uy^2 k~20
    //                  - ux^2 k~02 - 4 ux uy k~11 + ux uy (uy Fx + ux Fy)
    //                  - rho ux^2 uy^2
    // (the last from the expansion of sum f ex^2 ey^2 about u, with
    // k~10 = -Fx/2 and k~01 = -Fy/2), and their x <-> y images.
    const R cxy = kxy - uy * jx + ux * hFy;
    const R cxx = kxx - dr * third - ux * (jx - hFx);
    const R cyy = kyy - dr * third - uy * (jy - hFy);
    const R cxxy = kxxy - uy * (kxx + rt.r3) - ux2 * cxy + uxx * hFy;
    const R cxyy = kxyy - ux * (kyy + rt.r3) - uy2 * cxy + uyy * hFx;
    const R rho3 = rho * third;
    const R cxxyy = kxxyy - dr * ninth - uy2 * cxxy - ux2 * cxyy - uyy * (cxx + rho3) - uxx * (cyy + rho3) -
                    uxy * (R(4) * cxy + (uxy * rho - (uy * Fx + ux * Fy)));

    // Change of each central moment, Eq. (12) (or Eq. 21): the relaxation
    // -s (T~ - T~eq) and the force term; k~20 and k~02 relax as a trace
    // at sb and a deviator at s2.
    const R d20 = rt.nap * cxx + rt.nam * cyy;
    const R d02 = rt.nam * cxx + rt.nap * cyy;
    const R d11 = rt.ns2 * cxy;
    R d21, d12, d22, d10, d01;
    if (SCH == SCH_CONSISTENT) {
        // Eq. (14): C = [0, Fx, Fy, 0, 0, 0, Fy/3, Fx/3, 0].  The first-order
        // central moments go from -F/2 to +F/2 whatever s1 is.
        d10 = Fx;
        d01 = Fy;
        d21 = rt.ns3 * cxxy + rt.h3t * Fy;
        d12 = rt.ns3 * cxyy + rt.h3t * Fx;
        d22 = rt.ns4 * cxxyy;
    } else {
        // Eq. (21): central moments of Guo's term, weighted by 1 - s2/2; the
        // first-order slots relax at s1 from -F/2.
        d10 = rt.g1 * Fx;
        d01 = rt.g1 * Fy;
        d21 = rt.ns3 * cxxy + rt.h2 * (third * Fy - R(2) * uxy * Fx - uxx * Fy);
        d12 = rt.ns3 * cxyy + rt.h2 * (third * Fx - uyy * Fx - R(2) * uxy * Fy);
        d22 = rt.ns4 * cxxyy + rt.h2 * (R(4) * uxy * (uy * Fx + ux * Fy));
    }
    add_back<R>(g, ux, uy, d10, d01, d20, d02, d11, d21, d12, d22);
}

// Pre-collision deviations of the start state (central moments
// [rho, -Fx/2, -Fy/2, 2 rho/3, 0, 0, 0, 0, rho/9] about u).
template <typename R>
__host__ __device__ __forceinline__ void start_state(R rho0, R rho, R ux, R uy, R Fx, R Fy, R g[9])
{
    const R h = R(0.5);
    from_central<R>(rho - rho0, rho, rho * ux, rho * uy, ux, uy, -h * Fx, -h * Fy, R(0), R(0), R(0),
                    R(0), R(0), R(0), g);
}

}  // namespace clbm

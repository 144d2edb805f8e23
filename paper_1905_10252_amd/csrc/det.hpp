// Deterministic arithmetic used wherever a floating-point result decides an
// integer or feeds a bit-exact particle trajectory.  Every function is a fixed
// sequence of IEEE-754 binary64 operations (add, mul, fma, div, sqrt, rint,
// ldexp, frexp), so the device and any other faithful implementation of the
// same sequence agree bit for bit.  Compiled without FP contraction.
//
//   det_exp : Cody-Waite reduction x = k ln2 + r with the fdlibm two-part ln 2,
//             then e^r by its Taylor polynomial of degree 13 (Horner, fma),
//             then ldexp by k.  Domain of use: x <= 0.
//   det_log : x = m 2^e with m in [sqrt(1/2), sqrt(2)); log m = 2 atanh(f),
//             f = (m - 1)/(m + 1), odd series through f^23 (Horner in f^2,
//             fma); result e ln2_hi + (e ln2_lo + log m) with fma.
//   det_atan: |z| > 1 folded by atan z = pi/2 - atan(1/z); two halvings
//             a <- a / (1 + sqrt(1 + a^2)) (atan a = 2 atan of the result);
//             odd Taylor series of atan to a^25 by Horner in a^2 with fma;
//             times 4; pi/2 as a two-part constant.
//   Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and standard normals by
//   the Marsaglia-Bray polar method on its 53-bit uniforms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace smc {

// Horner coefficients.  kSc: on the device each coefficient reaches its fma
// through a scalar register pair (an empty asm statement with an SGPR
// operand).  An FP64 vector instruction cannot carry a 64-bit immediate, and
// left alone the compiler rebuilds every coefficient in vector registers with
// two vector moves per use; as a scalar operand it costs two scalar moves,
// which issue beside the vector work.  The value, and so every result, is the
// same either way.  The choice is made per call site: the scalar registers it
// takes are scarce in kernels that already hold many uniform values.
template <bool kSc>
__host__ __device__ inline double coef(double c)
{
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (kSc) {
        double r;
        asm volatile("" : "=s"(r) : "0"(c));
        return r;
    }
#endif
    return c;
}

template <bool kSc = false>
__host__ __device__ inline double det_exp(double x)
{
    if (x != x) return x;
    if (x < -746.0) return 0.0;
    if (x > 709.0) return __builtin_huge_val();
    const double kd = rint(x * 0x1.71547652b82fep+0);
    double r = fma(-kd, 0x1.62e42fee00000p-1, x);
    r = fma(-kd, 0x1.a39ef35793c76p-33, r);
    double p = coef<kSc>(0x1.6124613a86d09p-33);  // 1/13!
    p = fma(p, r, coef<kSc>(0x1.1eed8eff8d898p-29));  // 1/12!
    p = fma(p, r, coef<kSc>(0x1.ae64567f544e4p-26));  // 1/11!
    p = fma(p, r, coef<kSc>(0x1.27e4fb7789f5cp-22));  // 1/10!
    p = fma(p, r, coef<kSc>(0x1.71de3a556c734p-19));  // 1/9!
    p = fma(p, r, coef<kSc>(0x1.a01a01a01a01ap-16));  // 1/8!
    p = fma(p, r, coef<kSc>(0x1.a01a01a01a01ap-13));  // 1/7!
    p = fma(p, r, coef<kSc>(0x1.6c16c16c16c17p-10));  // 1/6!
    p = fma(p, r, coef<kSc>(0x1.1111111111111p-7));   // 1/5!
    p = fma(p, r, coef<kSc>(0x1.5555555555555p-5));   // 1/4!
    p = fma(p, r, coef<kSc>(0x1.5555555555555p-3));   // 1/3!
    p = fma(p, r, 0x1.0000000000000p-1);   // 1/2!
    p = fma(p, r, 1.0);                    // 1/1!
    p = fma(p, r, 1.0);                    // 1/0!
    return ldexp(p, (int)kd);
}

template <bool kSc = false>
__host__ __device__ inline double det_log(double x)
{
    if (!(x > 0.0)) return x == 0.0 ? -__builtin_huge_val() : __builtin_nan("");
    if (x == __builtin_huge_val()) return x;
    int e;
    double m = frexp(x, &e);
    if (m < 0x1.6a09e667f3bcdp-1) {
        m = m * 2.0;
        e = e - 1;
    }
    const double f = (m - 1.0) / (m + 1.0);
    const double s = f * f;
    double p = coef<kSc>(0x1.642c8590b2164p-4);   // 2/23
    p = fma(p, s, coef<kSc>(0x1.8618618618618p-4));  // 2/21
    p = fma(p, s, coef<kSc>(0x1.af286bca1af28p-4));  // 2/19
    p = fma(p, s, coef<kSc>(0x1.e1e1e1e1e1e1ep-4));  // 2/17
    p = fma(p, s, coef<kSc>(0x1.1111111111111p-3));  // 2/15
    p = fma(p, s, coef<kSc>(0x1.3b13b13b13b14p-3));  // 2/13
    p = fma(p, s, coef<kSc>(0x1.745d1745d1746p-3));  // 2/11
    p = fma(p, s, coef<kSc>(0x1.c71c71c71c71cp-3));  // 2/9
    p = fma(p, s, coef<kSc>(0x1.2492492492492p-2));  // 2/7
    p = fma(p, s, coef<kSc>(0x1.999999999999ap-2));  // 2/5
    p = fma(p, s, coef<kSc>(0x1.5555555555555p-1));  // 2/3
    p = fma(p, s, 2.0);                   // 2/1
    const double lm = f * p;
    const double E = (double)e;
    return fma(E, 0x1.62e42fee00000p-1, fma(E, 0x1.a39ef35793c76p-33, lm));
}

__host__ __device__ inline double det_sqrt(double v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __dsqrt_rn(v);
#else
    return __builtin_sqrt(v);
#endif
}

template <bool kSc = false>
__host__ __device__ inline double det_atan(double z)
{
    if (z != z) return z;
    const bool neg = z < 0.0;
    double a = neg ? -z : z;
    const bool inv = a > 1.0;
    if (inv) a = 1.0 / a;
    a = a / (1.0 + det_sqrt(fma(a, a, 1.0)));
    a = a / (1.0 + det_sqrt(fma(a, a, 1.0)));
    const double s = a * a;
    double p = coef<kSc>(0x1.47ae147ae147bp-5);      // 1/25
    p = fma(p, -s, coef<kSc>(0x1.642c8590b2164p-5));  // 1/23
    p = fma(p, -s, coef<kSc>(0x1.8618618618618p-5));  // 1/21
    p = fma(p, -s, coef<kSc>(0x1.af286bca1af28p-5));  // 1/19
    p = fma(p, -s, coef<kSc>(0x1.e1e1e1e1e1e1ep-5));  // 1/17
    p = fma(p, -s, coef<kSc>(0x1.1111111111111p-4));  // 1/15
    p = fma(p, -s, coef<kSc>(0x1.3b13b13b13b14p-4));  // 1/13
    p = fma(p, -s, coef<kSc>(0x1.745d1745d1746p-4));  // 1/11
    p = fma(p, -s, coef<kSc>(0x1.c71c71c71c71cp-4));  // 1/9
    p = fma(p, -s, coef<kSc>(0x1.2492492492492p-3));  // 1/7
    p = fma(p, -s, coef<kSc>(0x1.999999999999ap-3));  // 1/5
    p = fma(p, -s, coef<kSc>(0x1.5555555555555p-2));  // 1/3
    p = fma(p, -s, 1.0);                   // 1/1
    double r = 4.0 * (a * p);
    if (inv) r = (0x1.921fb54442d18p+0 - r) + 0x1.1a62633145c07p-54;
    return neg ? -r : r;
}

// ------------------------------------------------------------- Philox4x32-10
struct Philox4 {
    uint32_t v[4];
};

__host__ __device__ inline Philox4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                 uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t h0 = (uint32_t)(p0 >> 32), l0 = (uint32_t)p0;
        const uint32_t h1 = (uint32_t)(p1 >> 32), l1 = (uint32_t)p1;
        const uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{{c0, c1, c2, c3}};
}

// Random-number streams of the sampler.  Counter words: particle index,
// (pair << 16) | attempt, iteration, (stream tag << 24) | sampler id.
enum : uint32_t { kTagInit = 1, kTagPropose = 2, kTagResample = 3 };

__host__ __device__ inline Philox4 draw(uint64_t seed, uint32_t tag, uint32_t sampler, uint32_t t,
                                        uint32_t idx, uint32_t sub)
{
    return philox4x32_10(idx, sub, t, (tag << 24) | (sampler & 0xFFFFFFu), (uint32_t)seed,
                         (uint32_t)(seed >> 32));
}

// Two independent N(0,1) variates for pair `pair` of particle `idx`.
__host__ __device__ inline void normal_pair(uint64_t seed, uint32_t tag, uint32_t sampler,
                                            uint32_t t, uint32_t idx, uint32_t pair, double &z1,
                                            double &z2)
{
    for (uint32_t a = 0; a < 32u; ++a) {
        const Philox4 w = draw(seed, tag, sampler, t, idx, (pair << 16) | a);
        const uint64_t b1 = ((uint64_t)w.v[1] << 32) | w.v[0];
        const uint64_t b2 = ((uint64_t)w.v[3] << 32) | w.v[2];
        const double v1 = (double)(b1 >> 11) * 0x1p-52 - 1.0;
        const double v2 = (double)(b2 >> 11) * 0x1p-52 - 1.0;
        const double s = v1 * v1 + v2 * v2;
        if (s > 0.0 && s < 1.0) {
            const double c = (-2.0 * det_log(s)) / s;
            const double f = det_sqrt(c);
            z1 = v1 * f;
            z2 = v2 * f;
            return;
        }
    }
    z1 = 0.0;
    z2 = 0.0;
}

__host__ __device__ inline uint64_t resample_word(uint64_t seed, uint32_t sampler, uint32_t t)
{
    const Philox4 w = draw(seed, kTagResample, sampler, t, 0u, 0u);
    return ((uint64_t)w.v[1] << 32) | w.v[0];
}

}  // namespace smc

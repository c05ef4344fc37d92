// Device-side steps of quaternion-circle rotation voting for gfx950.
//
// Every floating-point operation here is one binary32 operation, round to
// nearest even.  The library is compiled with -ffp-contract=off and without
// fast-math, so the only fused multiply-adds are the explicit
// __builtin_fmaf calls, and '/' and sqrtf are the correctly rounded IEEE
// operations.  The fixed operation order is what lets the vote histogram be
// reproduced bit for bit by an independent implementation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rv {

constexpr int kWave = 64;

struct Quat {
    float w, x, y, z;
};

// Direction of one SoA vector (Sec. 4.1 works on unit a, b).  Returns false
// when the squared norm is not a positive finite float; the output is then a
// fixed unit vector so that later arithmetic stays finite.
__device__ __forceinline__ bool load_unit(const float* __restrict__ v, int64_t n, int64_t i,
                                          float out[3])
{
    const float v0 = v[i];
    const float v1 = v[n + i];
    const float v2 = v[2 * n + i];
    float s = v0 * v0;
    s = s + v1 * v1;
    s = s + v2 * v2;
    const float nrm = __builtin_sqrtf(s);
    const bool ok = (nrm > 0.0f) && (nrm < __builtin_inff());
    out[0] = ok ? v0 / nrm : 1.0f;
    out[1] = ok ? v1 / nrm : 0.0f;
    out[2] = ok ? v2 / nrm : 0.0f;
    return ok;
}

// Circle basis (Sec. 4.1, App. A).  M (q^T M q = b^T R(q) a) has eigenvalues
// (1,1,-1,-1); the rotations taking a to b are the unit vectors of its +1
// eigenspace, which contains every column of I + M.  The column k with the
// largest diagonal entry M_kk has squared norm 2 (1 + M_kk) >= 2 (trace M = 0),
// so it is normalised without a threshold.  Its entries are
//   M_00 = a.b, M_kk = 2 a_m b_m - a.b, M_k0 = (a x b)_m (k = m + 1),
//   M_{n+1,m+1} = a_n b_m + a_m b_n.
// The second vector v = (0, b) (x) u is the paper's q_b2 = q(alpha = pi).
__device__ __forceinline__ void circle_basis(const float a[3], const float b[3], Quat& u, Quat& v)
{
    const float p0 = a[0] * b[0];
    const float p1 = a[1] * b[1];
    const float p2 = a[2] * b[2];
    float d = p0 + p1;
    d = d + p2;
    const float c0 = a[1] * b[2] - a[2] * b[1];
    const float c1 = a[2] * b[0] - a[0] * b[2];
    const float c2 = a[0] * b[1] - a[1] * b[0];
    const float g1 = 2.0f * p0 - d;
    const float g2 = 2.0f * p1 - d;
    const float g3 = 2.0f * p2 - d;
    const float e01 = a[0] * b[1] + a[1] * b[0];
    const float e02 = a[0] * b[2] + a[2] * b[0];
    const float e12 = a[1] * b[2] + a[2] * b[1];

    // column k* = first index of max(d, g1, g2, g3)
    float uw = 1.0f + d, ux = c0, uy = c1, uz = c2, best = d;
    if (g1 > best) { best = g1; uw = c0; ux = 1.0f + g1; uy = e01; uz = e02; }
    if (g2 > best) { best = g2; uw = c1; ux = e01; uy = 1.0f + g2; uz = e12; }
    if (g3 > best) { best = g3; uw = c2; ux = e02; uy = e12; uz = 1.0f + g3; }

    float r2 = uw * uw;
    r2 = r2 + ux * ux;
    r2 = r2 + uy * uy;
    r2 = r2 + uz * uz;
    const float r = __builtin_sqrtf(r2);
    u.w = uw / r;
    u.x = ux / r;
    u.y = uy / r;
    u.z = uz / r;

    float bu = b[0] * u.x;
    bu = bu + b[1] * u.y;
    bu = bu + b[2] * u.z;
    v.w = -bu;
    v.x = u.w * b[0] + (b[1] * u.z - b[2] * u.y);
    v.y = u.w * b[1] + (b[2] * u.x - b[0] * u.z);
    v.z = u.w * b[2] + (b[0] * u.y - b[1] * u.x);
}

// Correctly rounded 1/d for d in [1, 2]: the hardware reciprocal (within one
// ulp) refined by one fused Newton step.  The test suite checks it against
// IEEE division for every binary32 value in [1, 2]; outside that range the
// caller must not use it.
__device__ __forceinline__ float recip_1_2(float d)
{
    const float r0 = __builtin_amdgcn_rcpf(d);
    const float e = __builtin_fmaf(-d, r0, 1.0f);
    return __builtin_fmaf(e, r0, r0);
}

// Canonical sign (Sec. 4.3: q and -q are one rotation; keep w >= 0 with the
// equator resolved by the first nonzero component), stereographic chart from
// the pole w = -1 (Sec. 4.3.1: p = q_vec / (1 + w)), and Alg. 1's cell of
// the cube [-1, 1]^3 at G steps per axis, x fastest.  The sign is folded into
// the chart scale: fma(-q_c, rh, H) == fma(q_c, -rh, H) exactly, and
// 1 + |w| is the canonical denominator in every case, w = -0 included.
struct Cell {
    unsigned x, y, z;
    unsigned y_b1;  // y << 8 when G <= 256 (see cell_coords); unused values cost nothing
    unsigned r8;    // x << 8 | y << 16 | z << 24 when G <= 256
};

template <bool kFastRecip>
__device__ __forceinline__ Cell cell_coords(float qw, float qx, float qy, float qz, float H, float gm)
{
    const float den = 1.0f + __builtin_fabsf(qw);
    const float r = kFastRecip ? recip_1_2(den) : 1.0f / den;
    const float rh = r * H;
    // w != 0: the sign of w decides; w = +-0: the first nonzero of x, y, z
    float srh = __builtin_copysignf(rh, qw);
    if (qw == 0.0f) {
        const bool neg = (qx != 0.0f) ? (qx < 0.0f) : ((qy != 0.0f) ? (qy < 0.0f) : (qz < 0.0f));
        srh = neg ? -rh : rh;
    }
    const float tx = __builtin_fmaf(qx, srh, H);
    const float ty = __builtin_fmaf(qy, srh, H);
    const float tz = __builtin_fmaf(qz, srh, H);
    // clamp(floor(t), 0, G-1) == trunc(med3(t, 0, G - 1/2)) for every finite t:
    // below 0 both give 0, on [0, G-1/2] trunc is floor, above both give G-1.
    Cell c;
    const float my = __builtin_amdgcn_fmed3f(ty, 0.0f, gm);
    c.x = (unsigned)__builtin_amdgcn_fmed3f(tx, 0.0f, gm);
    c.y = (unsigned)my;
    c.z = (unsigned)__builtin_amdgcn_fmed3f(tz, 0.0f, gm);
    // The same conversion written into byte 1 of a zeroed register: y << 8
    // for y < 256 in one instruction (the compiler only forms the word-1
    // variant by itself).
    asm("v_cvt_u32_f32_sdwa %0, %1 dst_sel:BYTE_1 dst_unused:UNUSED_PAD src0_sel:DWORD"
        : "=v"(c.y_b1)
        : "v"(my));
    // The cell one byte per axis in bytes 1-3 (G <= 256; byte 0 free for a
    // run length): x converted into byte 1 of a zeroed register, y and z into
    // bytes 2 and 3 of the same register, its other bytes kept.
    unsigned r8;
    asm("v_cvt_u32_f32_sdwa %0, %1 dst_sel:BYTE_1 dst_unused:UNUSED_PAD src0_sel:DWORD"
        : "=v"(r8)
        : "v"(__builtin_amdgcn_fmed3f(tx, 0.0f, gm)));
    asm("v_cvt_u32_f32_sdwa %0, %1 dst_sel:BYTE_2 dst_unused:UNUSED_PRESERVE src0_sel:DWORD"
        : "+v"(r8)
        : "v"(my));
    asm("v_cvt_u32_f32_sdwa %0, %1 dst_sel:BYTE_3 dst_unused:UNUSED_PRESERVE src0_sel:DWORD"
        : "+v"(r8)
        : "v"(__builtin_amdgcn_fmed3f(tz, 0.0f, gm)));
    c.r8 = r8;
    return c;
}

// Linear cell index, x fastest; G <= 1024 keeps every factor in 24 bits.
__device__ __forceinline__ unsigned linear_index(const Cell& c, unsigned G)
{
    return __umul24(__umul24(c.z, G) + c.y, G) + c.x;
}

// Cell coordinates packed 8 bits each (G <= 256) or 9 bits each (G <= 512):
// a key that is unique per cell and cheap to build and to take apart.
template <bool kWide = false>
__device__ __forceinline__ unsigned packed_coords(const Cell& c)
{
    constexpr int kBits = kWide ? 9 : 8;
    if constexpr (!kWide)
        return c.x | c.y_b1 | (c.z << 16);
    return c.x | (c.y << kBits) | (c.z << (2 * kBits));
}

template <bool kFastRecip>
__device__ __forceinline__ int cell_index(float qw, float qx, float qy, float qz, float H, float gm,
                                          int G)
{
    return (int)linear_index(cell_coords<kFastRecip>(qw, qx, qy, qz, H, gm), (unsigned)G);
}

// Sample j of the circle: q = cos(theta_j) u + sin(theta_j) v, per component
// fma(C, u_c, S * v_c) (Alg. 1, q(alpha) with theta = alpha / 2).
template <bool kFastRecip>
__device__ __forceinline__ Cell sample_cell(const Quat& u, const Quat& v, float C, float S, float H,
                                            float gm)
{
    const float qw = __builtin_fmaf(C, u.w, S * v.w);
    const float qx = __builtin_fmaf(C, u.x, S * v.x);
    const float qy = __builtin_fmaf(C, u.y, S * v.y);
    const float qz = __builtin_fmaf(C, u.z, S * v.z);
    return cell_coords<kFastRecip>(qw, qx, qy, qz, H, gm);
}

// Calls f(cell, j) for the samples j in [ja, jb) of the circle (u, v).  The
// (cos, sin) table index is wave-uniform, so the table is read with scalar
// loads, eight entries at a time; ja must be a multiple of 8.
template <bool kFastRecip, class F>
__device__ __forceinline__ void for_samples(const Quat& u, const Quat& v,
                                            const float2* __restrict__ table, int ja, int jb,
                                            float H, float gm, F&& f)
{
    const float4* __restrict__ t4 = reinterpret_cast<const float4*>(table);
    int j = ja;
    for (; j + 8 <= jb; j += 8) {
        const float4 c0 = t4[(j >> 1) + 0];
        const float4 c1 = t4[(j >> 1) + 1];
        const float4 c2 = t4[(j >> 1) + 2];
        const float4 c3 = t4[(j >> 1) + 3];
        f(sample_cell<kFastRecip>(u, v, c0.x, c0.y, H, gm), j + 0);
        f(sample_cell<kFastRecip>(u, v, c0.z, c0.w, H, gm), j + 1);
        f(sample_cell<kFastRecip>(u, v, c1.x, c1.y, H, gm), j + 2);
        f(sample_cell<kFastRecip>(u, v, c1.z, c1.w, H, gm), j + 3);
        f(sample_cell<kFastRecip>(u, v, c2.x, c2.y, H, gm), j + 4);
        f(sample_cell<kFastRecip>(u, v, c2.z, c2.w, H, gm), j + 5);
        f(sample_cell<kFastRecip>(u, v, c3.x, c3.y, H, gm), j + 6);
        f(sample_cell<kFastRecip>(u, v, c3.z, c3.w, H, gm), j + 7);
    }
    for (; j < jb; ++j) {
        const float2 cs = table[j];
        f(sample_cell<kFastRecip>(u, v, cs.x, cs.y, H, gm), j);
    }
}

// Loads correspondence i (if i < n) and builds its circle basis.  Unusable or
// absent correspondences get the basis of a = b = e_x and report false.
__device__ __forceinline__ bool load_circle(const float* __restrict__ x, const float* __restrict__ y,
                                            int64_t n, int64_t i, Quat& u, Quat& v)
{
    float a[3] = {1.0f, 0.0f, 0.0f};
    float b[3] = {1.0f, 0.0f, 0.0f};
    bool ok = false;
    if (i < n) {
        const bool oka = load_unit(x, n, i, a);
        const bool okb = load_unit(y, n, i, b);
        ok = oka && okb;
    }
    if (!ok) {
        a[0] = 1.0f; a[1] = 0.0f; a[2] = 0.0f;
        b[0] = 1.0f; b[1] = 0.0f; b[2] = 0.0f;
    }
    circle_basis(a, b, u, v);
    return ok;
}

__device__ __forceinline__ void canonical(Quat& q)
{
    const bool neg = (q.w != 0.0f) ? (q.w < 0.0f)
                   : (q.x != 0.0f) ? (q.x < 0.0f)
                   : (q.y != 0.0f) ? (q.y < 0.0f)
                                   : (q.z < 0.0f);
    if (neg) {
        q.w = -q.w;
        q.x = -q.x;
        q.y = -q.y;
        q.z = -q.z;
    }
}

// Cell centre back to the sphere (inverse of the chart, Sec. 4.3.1):
// w = (1 - s) / (1 + s), q_vec = 2 p / (1 + s), s = |p|^2.
__device__ __forceinline__ Quat decode_cell(int idx, int G)
{
    const int ix = idx % G;
    const int iy = (idx / G) % G;
    const int iz = idx / (G * G);
    const float fg = (float)G;
    const float px = (float)(2 * ix + 1) / fg - 1.0f;
    const float py = (float)(2 * iy + 1) / fg - 1.0f;
    const float pz = (float)(2 * iz + 1) / fg - 1.0f;
    float s = px * px;
    s = s + py * py;
    s = s + pz * pz;
    const float den = 1.0f + s;
    Quat q;
    q.w = (1.0f - s) / den;
    q.x = (2.0f * px) / den;
    q.y = (2.0f * py) / den;
    q.z = (2.0f * pz) / den;
    canonical(q);
    return q;
}

// Squared residual |L(a, b) q|^2 of App. D's constraint
// L = [0, (a-b)^T; -(a-b), [a+b]_x]; equals |R(q) a - b|^2 for unit q.
__device__ __forceinline__ float residual2(const float D[3], const float P[3], const Quat& q)
{
    float r0 = D[0] * q.x;
    r0 = r0 + D[1] * q.y;
    r0 = r0 + D[2] * q.z;
    const float r1 = (P[1] * q.z - P[2] * q.y) - q.w * D[0];
    const float r2 = (P[2] * q.x - P[0] * q.z) - q.w * D[1];
    const float r3 = (P[0] * q.y - P[1] * q.x) - q.w * D[2];
    float s = r0 * r0;
    s = s + r1 * r1;
    s = s + r2 * r2;
    s = s + r3 * r3;
    return s;
}

}  // namespace rv

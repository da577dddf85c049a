// Device-side B-spline primitives for gfx950 (FP32).
//
// Rows a2 (knot-span search) and a3 (basis and first derivative) of the
// decode/query path.  The paper hands micro-model evaluation to an MFA
// tensor-product B-spline (Sec. 4.2) and queries value and gradient per
// sample (Alg. 4); de Boor's recursion (the spline basis cited in Sec. 1)
// defines the basis.  Here it is evaluated in the triangular left/right
// form: only the p+1 functions that are non-zero on the span are built,
// degree by degree, every denominator being a sum of two knot distances
// that is positive on a non-empty span, so no zero test is needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fa.h"

namespace fa {

constexpr int kWave = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int kMaxKnotsPerBlock = 3 * (FA_MAX_NCP + FA_MAX_DEGREE + 1);

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Largest s in [p, n-1] with t[s] <= u, for u in [0, 1]; u >= t[n] (= 1)
// gives n-1.  Binary search keeping t[lo] <= u < t[hi].
template <typename KP>
__device__ __forceinline__ int span_search(int n, int p, KP t, float u) {
    if (u >= t[n]) return n - 1;
    int lo = p, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (u < t[mid]) hi = mid;
        else lo = mid;
    }
    return lo;
}

// Span from a first guess: walk down/up until t[s] <= u < t[s+1].  For
// uniform knots the guess p + floor(u (n-p)) is off by at most one, so the
// walk costs two comparisons against the stored knots.
template <typename KP>
__device__ __forceinline__ int span_from_guess(int n, int p, KP t, float u, int s) {
    s = s < p ? p : (s > n - 1 ? n - 1 : s);
    while (s > p && u < t[s]) --s;
    while (s < n - 1 && u >= t[s + 1]) ++s;
    return s;
}

// N[r] = N_{s-P+r,P}(u), D[r] = N'_{s-P+r,P}(u), r = 0..P.
template <int P, typename KP>
__device__ __forceinline__ void basis_ders(KP t, int s, float u, float (&N)[P + 1],
                                           float (&D)[P + 1]) {
    // no fused operations: the values do not depend on how the compiler
    // contracts the code it is inlined into (kernels that must agree bit
    // for bit, such as the decode and its residual form, share them)
#pragma clang fp contract(off)
    float left[P + 1], right[P + 1], low[P + 1];
    N[0] = 1.0f;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
        left[k] = u - t[s + 1 - k];
        right[k] = t[s + k] - u;
        if (k == P) {
#pragma unroll
            for (int r = 0; r < P; ++r) low[r] = N[r];  // degree P-1 values
        }
        float saved = 0.0f;
#pragma unroll
        for (int r = 0; r < k; ++r) {
            float q = N[r] * rcp(right[r + 1] + left[k - r]);
            N[r] = saved + right[r + 1] * q;
            saved = left[k - r] * q;
        }
        N[k] = saved;
    }
    // N'_{i,P} = P N_{i,P-1}/(t_{i+P}-t_i) - P N_{i+1,P-1}/(t_{i+P+1}-t_{i+1}),
    // i = s-P+r; the degree P-1 function N_{s-P+1+m} is low[m].
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        float d = 0.0f;
        if (r >= 1) d += low[r - 1] * rcp(t[s + r] - t[s - P + r]);
        if (r <= P - 1) d -= low[r] * rcp(t[s + r + 1] - t[s - P + r + 1]);
        D[r] = float(P) * d;
    }
}

// basis_ders<P> on a knot window held in registers: tw[m] = t[s-P+1+m],
// m = 0..2P-1 (every knot the p+1 non-zero functions and their
// derivatives touch), so all indices are compile-time constants.  The
// derivative's denominators t[s+m] - t[s+m-P] (m = 1..P) are the ones of
// the recursion's last degree, so their reciprocals are reused: P(P+1)/2
// reciprocals per axis instead of P(P+1)/2 + 2P.
template <int P>
__device__ __forceinline__ void basis_ders_win(const float (&tw)[2 * P], float u,
                                               float (&N)[P + 1], float (&D)[P + 1]) {
    // explicit fused operations only: every code path that inlines this
    // computes bit-identical values
#pragma clang fp contract(off)
    float left[P + 1], right[P + 1], low[P + 1], inv[P + 1];
    N[0] = 1.0f;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
        left[k] = u - tw[P - k];       // u - t[s+1-k]
        right[k] = tw[P - 1 + k] - u;  // t[s+k] - u
        if (k == P) {
#pragma unroll
            for (int r = 0; r < P; ++r) low[r] = N[r];
        }
        float saved = 0.0f;
#pragma unroll
        for (int r = 0; r < k; ++r) {
            const float iv = rcp(right[r + 1] + left[k - r]);  // 1 / (t[s+r+1] - t[s+r+1-k])
            if (k == P) inv[r + 1] = iv;
            const float q = N[r] * iv;
            N[r] = fmaf(right[r + 1], q, saved);
            saved = left[k - r] * q;
        }
        N[k] = saved;
    }
    // N'_{i,P} = P N_{i,P-1}/(t_{i+P}-t_i) - P N_{i+1,P-1}/(t_{i+P+1}-t_{i+1}),
    // i = s-P+r: the denominators are t[s+r] - t[s+r-P] = 1/inv[r] and
    // t[s+r+1] - t[s+r+1-P] = 1/inv[r+1].
#pragma unroll
    for (int r = 0; r <= P; ++r) {
        float d = 0.0f;
        if (r >= 1) d = low[r - 1] * inv[r];
        if (r <= P - 1) d = fmaf(-low[r], inv[r + 1], d);
        D[r] = float(P) * d;
    }
}

// Same as basis_ders<P> for a run-time degree p <= 3; entries beyond p are
// zero.  One instantiation serves every degree (used where the window is
// zero padded anyway, as in the dense matrix-core contraction).
__device__ __forceinline__ void basis_ders_rt(const float *t, int s, float u, int p,
                                              float (&N)[4], float (&D)[4]) {
#pragma clang fp contract(off)
    float left[4] = {0, 0, 0, 0}, right[4] = {0, 0, 0, 0}, low[4] = {0, 0, 0, 0};
    N[0] = 1.0f;
    N[1] = N[2] = N[3] = 0.0f;
#pragma unroll
    for (int k = 1; k <= 3; ++k) {
        if (k > p) break;
        left[k] = u - t[s + 1 - k];
        right[k] = t[s + k] - u;
        if (k == p) {
#pragma unroll
            for (int r = 0; r < 3; ++r) low[r] = N[r];
        }
        float saved = 0.0f;
#pragma unroll
        for (int r = 0; r < k; ++r) {
            float q = N[r] * rcp(right[r + 1] + left[k - r]);
            N[r] = saved + right[r + 1] * q;
            saved = left[k - r] * q;
        }
        N[k] = saved;
    }
#pragma unroll
    for (int r = 0; r <= 3; ++r) {
        float d = 0.0f;
        if (r <= p) {
            if (r >= 1) d += low[r - 1] * rcp(t[s + r] - t[s - p + r]);
            if (r <= p - 1) d -= low[r] * rcp(t[s + r + 1] - t[s - p + r + 1]);
        }
        D[r] = float(p) * d;
    }
}

// Raw buffer resource over `bytes` bytes at a wave-uniform base (gfx9
// word 3: 32-bit data format, no swizzle).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, uint32_t bytes) {
    const uint64_t v = reinterpret_cast<uint64_t>(base);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    void *p = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    return __builtin_amdgcn_make_buffer_rsrc(p, (short)0, (int)bytes, 0x00020000);
}

// Workgroup barrier for LDS hand-offs only: orders LDS accesses around
// s_barrier without waiting for outstanding global loads and stores (which
// __syncthreads() would drain), so prefetches and output stores stay in
// flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// XCD-aware workgroup order.  The dispatcher deals workgroups round-robin
// over the 8 XCDs (workgroup b runs on XCD b % 8), each with its own L2.
// This maps b to a logical index so that the workgroups one XCD runs are
// consecutive logical indices; when consecutive indices touch neighbouring
// data, each XCD's L2 then holds one compact region instead of a share of
// everything.  A permutation of [0, n) for any n.
constexpr int kXcds = 8;

__device__ __forceinline__ int xcd_order(int b, int n) {
    const int q = n / kXcds, r = n % kXcds;  // XCD x runs q + (x < r) workgroups
    const int x = b % kXcds, k = b / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Grid position of voxel i on an axis of resolution R (FP32, correctly
// rounded quotient; both sides of a parity check use this exact value).
__device__ __forceinline__ float grid_pos(int i, int R) {
    return __fdiv_rn(float(i), float(R - 1));
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(uint32_t(h) << 16);
}

__device__ __forceinline__ float f16_to_f32(uint16_t h) {
    _Float16 x;
    __builtin_memcpy(&x, &h, 2);
    return float(x);
}

// One control point of any storage type, as FP32 (scale applied to the
// 2-byte types).
__device__ __forceinline__ float load_ctrl(const void *ctrl, int dtype, int64_t idx, float scale) {
    if (dtype == FA_F32) return static_cast<const float *>(ctrl)[idx];
    uint16_t h = static_cast<const uint16_t *>(ctrl)[idx];
    return (dtype == FA_BF16 ? bf16_to_f32(h) : f16_to_f32(h)) * scale;
}

}  // namespace fa

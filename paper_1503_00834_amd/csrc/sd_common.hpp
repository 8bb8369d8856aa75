// Index helpers and 1D operator tables shared by the FP64 and mixed
// precision SD kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "chorus_internal.hpp"

namespace chorus {

// 1D SD operators of order N in arithmetic type T
template <typename T, int N>
struct OpsT {
    T I[N + 1][N];  // I[m][s] = h_s(xf[m])
    T D[N][N + 1];  // D[s][m] = l_m'(xs[s])
    T B[N][N];      // sum_{m=1}^{N-1} D[s][m] I[m][s']: interior flux points folded
};
template <int N>
using Ops = OpsT<double, N>;

template <typename T, int N>
inline OpsT<T, N> make_ops_t(const Basis1D &b) {
    OpsT<T, N> o;
    for (int m = 0; m <= N; ++m)
        for (int s = 0; s < N; ++s) o.I[m][s] = (T)b.I[m][s];
    for (int s = 0; s < N; ++s)
        for (int m = 0; m <= N; ++m) o.D[s][m] = (T)b.D[s][m];
    for (int a = 0; a < N; ++a)
        for (int s = 0; s < N; ++s) {
            double v = 0.0;
            for (int m = 1; m < N; ++m) v += b.D[a][m] * b.I[m][s];
            o.B[a][s] = (T)v;
        }
    return o;
}



// Copy the 1D operator tables into LDS.  Kernels index them with per-lane
// indices, which on a by-value kernel argument compile to vector loads from
// the argument segment on every line operation.  Each lane copies one word
// (one vector load from the argument segment per lane, once per block: a
// copy by one lane from scalar registers issues one vector instruction per
// word); the caller's first barrier publishes the tables.
template <typename T, int N>
__device__ __forceinline__ void ops_to_lds(const OpsT<T, N> &src, OpsT<T, N> &dst) {
    constexpr int NW = (int)(sizeof(OpsT<T, N>) / sizeof(uint32_t));
    static_assert(sizeof(OpsT<T, N>) % sizeof(uint32_t) == 0, "tables of words");
    const uint32_t *s = reinterpret_cast<const uint32_t *>(&src);
    uint32_t *d = reinterpret_cast<uint32_t *>(&dst);
    for (int i = threadIdx.x; i < NW; i += blockDim.x) d[i] = s[i];
}

// line through solution point (a along d; t1 < t2 the tangential indices).
// Written with arithmetic selects: d is often lane dependent (face points),
// and nested conditionals on it compiled to divergent branches recomputed
// for every field.
template <int N>
__device__ __forceinline__ int stride_of(int d) {
    return (d == 0) ? 1 : ((d == 1) ? N : N * N);
}
template <int N>
__device__ __forceinline__ int sol_of(int d, int a, int t1, int t2) {
    const int s1 = (d == 0) ? N : 1, s2 = (d == 2) ? N : N * N;
    return a * stride_of<N>(d) + t1 * s1 + t2 * s2;
}
template <int N>
__device__ __forceinline__ void split_sol(int d, int p, int &a, int &t1, int &t2) {
    const int i = p % N, j = (p / N) % N, k = p / (N * N);
    if (d == 0) { a = i; t1 = j; t2 = k; }
    else if (d == 1) { a = j; t1 = i; t2 = k; }
    else { a = k; t1 = i; t2 = j; }
}
template <int N>
__device__ __forceinline__ int map_face_point(int o, int t1, int t2) {
    int u1 = (o & 4) ? t2 : t1, u2 = (o & 4) ? t1 : t2;
    if (o & 2) u1 = N - 1 - u1;
    if (o & 1) u2 = N - 1 - u2;
    return u1 + N * u2;
}

// Global access at a base pointer plus a small per-lane offset in elements
// (its byte offset fits 32 bits).  With a block-uniform base the address is
// a scalar base plus a 32-bit vector offset: no 64-bit vector arithmetic per
// access.
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t i) {
    return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + i * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_off(T *base, uint32_t i, T v) {
    *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + i * (uint32_t)sizeof(T)) = v;
}

// access of data touched once per pass (mailboxes, geometry): the
// non-temporal hint lets it leave the caches first
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

// LDS slot of solution point p in an element's FP64 field array.  A line
// operator reads one lattice plane per instruction (the points of all lines
// of one direction at one position along them); at order 4 the in-plane
// index is XORed with 5 k (k the third lattice index), so that the 16
// points of every plane occupy distinct 8-byte bank pairs modulo 16 and
// modulo 32.  Other orders keep the natural index.
template <int N>
__device__ __forceinline__ int lds_sol(int p) {
    if constexpr (N == 4) return p ^ ((p >> 4) * 5);
    else return p;
}
// slot of point b of the line (base, st) (base at lattice index 0 along the
// line): lds_sol is linear over XOR and base and b st share no set bit, so
// the per-line part is computed once and the rest is a constant
template <int N>
__device__ __forceinline__ int lds_line(int base, int b, int st) {
    if constexpr (N == 4) return lds_sol<N>(base) ^ lds_sol<N>(b * st);
    else return base + b * st;
}

// mailbox slot of face point pp of an element's face (nb, inf = the face's
// neighbour element and info word): the receiving element's face and point
// (the orientation map applied), first variable; the next is NF2 further on
// (NV variables per face point)
template <int N, int NV = 5>
__device__ __forceinline__ int64_t mailbox_slot(int32_t nb, int32_t inf, int pp) {
    constexpr int NF2 = N * N;
    const int f2 = inf & 7, o = (inf >> 3) & 7;
    const int pn = map_face_point<N>(o, pp % N, pp / N);
    return ((int64_t)nb * 6 + f2) * NV * NF2 + pn;
}

}  // namespace chorus

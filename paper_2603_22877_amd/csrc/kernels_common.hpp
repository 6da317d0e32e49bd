// Device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fsmt_internal.hpp"

namespace fsmt {

// Address-space-typed device pointers. Kernels find their tables and state through
// descriptors in device memory; plain pointers read from there would be generic to the
// compiler (flat loads), and it could not tell that the tables are never written.
//   cptr: data that no kernel of the launch writes (constant address space: loads at
//         wave-uniform addresses become scalar loads, the others global loads);
//   gptr: read-write global memory.
// Host code fills both with an explicit cast of a device allocation.
template <class T> using cptr = const __attribute__((address_space(4))) T *;
template <class T> using gptr = __attribute__((address_space(1))) T *;
template <class T> using gref = __attribute__((address_space(1))) T &;
template <class T> inline cptr<T> as_cptr(const T *p) { return (cptr<T>)p; }
template <class T> inline gptr<T> as_gptr(T *p) { return (gptr<T>)p; }

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));

// Strided [rows][cols] float view (see fsmt_view).
struct View {
    gptr<float> data = nullptr;
    int32_t rows = 0, cols = 0;
    int64_t sr = 0, sv = 0;
    __device__ __forceinline__ gref<float> at(int r, int j) const { return data[(int64_t)r * sr + (int64_t)j * sv]; }
    static View of(const fsmt_view &v) { return View{as_gptr(v.data), v.rows, v.cols, v.stride_r, v.stride_v}; }
};

// Hardware float atomic add in L2 (global_atomic_add_f32) on coarse-grained device memory.
__device__ __forceinline__ void atomic_add_f32(gptr<float> p, float v) { unsafeAtomicAdd((float *)p, v); }
__device__ __forceinline__ void atomic_add_f32(float *p, float v) { unsafeAtomicAdd(p, v); }

// Index of this thread's wavefront in the block, as a wave-uniform (scalar) value: the
// compiler does not know that threadIdx.x / 64 is uniform across a wave64.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Node record at a wave-uniform address (a scalar load); its fields are marked uniform so
// that the message arrays are indexed with scalar indices.
__device__ __forceinline__ Node load_node(cptr<Node> p) {
    const u32x2 raw = *(cptr<u32x2>)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane(raw.x), hi = __builtin_amdgcn_readfirstlane(raw.y);
    Node n;
    n.slot = (uint16_t)(lo & 0xFFFFu);
    n.hi = (uint16_t)(lo >> 16);
    n.lo = (uint16_t)(hi & 0xFFFFu);
    n.pad = 0;
    return n;
}

// Node record at a per-lane address (a vector load).
__device__ __forceinline__ Node load_node_lane(cptr<Node> p) {
    const u32x2 raw = *(cptr<u32x2>)p;
    Node n;
    n.slot = (uint16_t)(raw.x & 0xFFFFu);
    n.hi = (uint16_t)(raw.x >> 16);
    n.lo = (uint16_t)(raw.y & 0xFFFFu);
    n.pad = 0;
    return n;
}

// Bucket record (64 bytes; one s_load_dwordx16 at a wave-uniform address).
__device__ __forceinline__ BucketInfo load_bucket(cptr<BucketInfo> p) {
    static_assert(sizeof(BucketInfo) == 64, "bucket record layout");
    const i32x16 raw = *(cptr<i32x16>)p;
    BucketInfo b;
    __builtin_memcpy(&b, &raw, sizeof(b));
    return b;
}

// Sum over a block of up to 1024 threads (result valid in every thread).
__device__ __forceinline__ float block_sum(float v) {
    __shared__ float part[16];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part[w] = v;
    __syncthreads();
    float t = 0.0f;
    for (int i = 0; i < nw; ++i) t += part[i];
    __syncthreads();
    return t;
}

// Half-spaces q.y <= rhs of the feasible set (multi-variable unit atoms), stored by colour
// class: the half-spaces cstart[k] .. cstart[k+1]-1 share no variable.
struct HalfSpaces {
    cptr<int32_t> ptr, var;
    cptr<float> coef, rhs, inv;
    cptr<int32_t> cstart;
    int32_t n, nnz, n_colors;
    int32_t separable;   // no shared variable, few distinct variables per row: closed form
};

// Orders this wave's LDS accesses (the next instructions read what this wave wrote).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xc07f);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ float clip_to(float z, float l, float h) { return z < l ? l : (z > h ? h : z); }

// Projection onto the box and half-spaces that share no variable, each over at most
// kSeparableRowMax distinct variables (hs.separable). The problem separates into one
// projection per half-space onto {x in its variables' box : a.x <= r}; the other variables
// are only clipped. By the KKT conditions that projection is clip(y - lam a) with lam >= 0
// the root of g(lam) = a.clip(y - lam a) - r when g(0) > 0. g does not increase and is
// linear between its breakpoints (where a coordinate reaches a bound), so the root lies on
// the segment between the last breakpoint with g > 0 and the first with g <= 0. If g stays
// positive the half-space misses the box; its point of least excess (every coordinate at
// the bound minimizing a.x) is taken. One lane per half-space, its row in registers.
__device__ __forceinline__ void project_separable(float *y, float *pb, cptr<float> lo, cptr<float> hi, int m,
                                                  const HalfSpaces &hs) {
    constexpr int K = kSeparableRowMax;
    for (int j = threadIdx.x; j < m; j += blockDim.x) pb[j] = clip_to(y[j], lo[j], hi[j]);
    __syncthreads();
    for (int t = threadIdx.x; t < hs.n; t += blockDim.x) {
        const int e0 = hs.ptr[t], ne = hs.ptr[t + 1] - e0;
        const float r = hs.rhs[t];
        int jv[K];
        float av[K], yv[K], lv[K], hv[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            jv[q] = 0;
            av[q] = 0.0f;
            if (q < ne) {
                jv[q] = hs.var[e0 + q];
                av[q] = hs.coef[e0 + q];
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            yv[q] = lv[q] = hv[q] = 0.0f;   // padding: a = 0 adds nothing to g
            if (q < ne) {
                yv[q] = y[jv[q]];
                lv[q] = lo[jv[q]];
                hv[q] = hi[jv[q]];
            }
        }
        auto excess = [&](float lam) {
            float g = -r;
#pragma unroll
            for (int q = 0; q < K; ++q) g += av[q] * clip_to(yv[q] - lam * av[q], lv[q], hv[q]);
            return g;
        };
        const float g0 = excess(0.0f);
        if (!(g0 > 0.0f)) continue;
        float L = 0.0f, gL = g0, U = INFINITY, gU = 0.0f;
#pragma unroll
        for (int q = 0; q < K; ++q) {
            if (q >= ne || av[q] == 0.0f) continue;
            for (int s = 0; s < 2; ++s) {
                const float bp = (yv[q] - (s ? hv[q] : lv[q])) / av[q];
                if (!(bp > 0.0f)) continue;
                const float g = excess(bp);
                if (g > 0.0f) {
                    if (bp > L) { L = bp; gL = g; }
                } else if (bp < U) {
                    U = bp;
                    gU = g;
                }
            }
        }
        const float lam = U == INFINITY ? L : L + gL * ((U - L) / (gL - gU));
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q < ne) pb[jv[q]] = clip_to(yv[q] - lam * av[q], lv[q], hv[q]);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < m; j += blockDim.x) y[j] = pb[j];
    __syncthreads();
}

// Euclidean projection of y[0..m) (LDS) onto [lo, hi] intersected with the half-spaces
// (Prop. "qp"). Half-spaces that share no variable and have few variables each
// (hs.separable) are solved in closed form (project_separable). Otherwise: if the clamped
// point already satisfies every half-space it is the projection; else Dykstra's alternating
// projections run from y (the colour classes of half-spaces in order, then the box, per
// sweep; increments pb[m], ph[nnz] in LDS) until a sweep moves no coordinate by more than
// 4e-7 (1 + |y|), or 256 sweeps. Projecting onto a class is projecting onto each member
// independently (they share no variable), so the members of a class run on parallel lanes.
// The sweeps run on the block's first wavefront alone, ordered by LDS waits instead of
// block barriers. All threads of the block must call it.
__device__ __forceinline__ void project_dykstra(float *y, float *pb, float *ph, cptr<float> lo, cptr<float> hi,
                                                int m, const HalfSpaces &hs) {
    if (hs.separable) {
        project_separable(y, pb, lo, hi, m, hs);
        return;
    }
    for (int j = threadIdx.x; j < m; j += blockDim.x) pb[j] = y[j] < lo[j] ? lo[j] : (y[j] > hi[j] ? hi[j] : y[j]);
    __syncthreads();
    int violated = 0;
    for (int t = threadIdx.x; t < hs.n; t += blockDim.x) {
        float v = -hs.rhs[t];
        for (int e = hs.ptr[t]; e < hs.ptr[t + 1]; ++e) v += hs.coef[e] * pb[hs.var[e]];
        violated |= v > 0.0f ? 1 : 0;
    }
    if (!__syncthreads_or(violated)) {
        for (int j = threadIdx.x; j < m; j += blockDim.x) y[j] = pb[j];
        __syncthreads();
        return;
    }
    if (threadIdx.x < 64) {
        const int lane = threadIdx.x;
        for (int j = lane; j < m; j += 64) pb[j] = 0.0f;
        for (int e = lane; e < hs.nnz; e += 64) ph[e] = 0.0f;
        wave_lds_sync();
        for (int sweep = 0; sweep < 256; ++sweep) {
            int moved = 0;
            for (int k = 0; k < hs.n_colors; ++k) {
                for (int t = hs.cstart[k] + lane; t < hs.cstart[k + 1]; t += 64) {
                    const int e0 = hs.ptr[t], e1 = hs.ptr[t + 1];
                    float viol = -hs.rhs[t];
                    for (int e = e0; e < e1; ++e) viol += hs.coef[e] * (y[hs.var[e]] + ph[e]);
                    const float sh = viol > 0.0f ? viol * hs.inv[t] : 0.0f;
                    for (int e = e0; e < e1; ++e) {
                        const int j = hs.var[e];
                        const float z = y[j] + ph[e], yp = z - sh * hs.coef[e];
                        if (fabsf(yp - y[j]) > 4e-7f * (1.0f + fabsf(yp))) moved = 1;
                        ph[e] = z - yp;
                        y[j] = yp;
                    }
                }
                wave_lds_sync();
            }
            for (int j = lane; j < m; j += 64) {
                const float z = y[j] + pb[j];
                const float yp = z < lo[j] ? lo[j] : (z > hi[j] ? hi[j] : z);
                if (fabsf(yp - y[j]) > 4e-7f * (1.0f + fabsf(yp))) moved = 1;
                pb[j] = z - yp;
                y[j] = yp;
            }
            wave_lds_sync();
            if (__ballot(moved) == 0) break;
        }
    }
    __syncthreads();
}

// Sums of two values over the block (results valid in every thread).
__device__ __forceinline__ float2 block_sum2(float a, float b) {
    __shared__ float2 part2[16];
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) part2[w] = make_float2(a, b);
    __syncthreads();
    float2 t = make_float2(0.0f, 0.0f);
    for (int i = 0; i < nw; ++i) {
        t.x += part2[i].x;
        t.y += part2[i].y;
    }
    return t;
}

fsmt_status fill_view(const fsmt_view &v, float value, hipStream_t st);
fsmt_status fill_f32(float *p, int64_t n, float value, hipStream_t st);
fsmt_status fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t st);
fsmt_status check_device_ptr(const void *p, int device, const char *name);
fsmt_status select_device(const fsmt_xbdd *h);
HalfSpaces halfspaces_of(const fsmt_xbdd *h);

}  // namespace fsmt

// Device helpers shared by the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fsmt_internal.hpp"

namespace fsmt {

// Strided [rows][cols] float view (see fsmt_view).
struct View {
    float *data = nullptr;
    int32_t rows = 0, cols = 0;
    int64_t sr = 0, sv = 0;
    __host__ __device__ __forceinline__ float &at(int r, int j) const { return data[(int64_t)r * sr + (int64_t)j * sv]; }
    static View of(const fsmt_view &v) { return View{v.data, v.rows, v.cols, v.stride_r, v.stride_v}; }
};

// Hardware float atomic add in L2 (global_atomic_add_f32) on coarse-grained device memory.
__device__ __forceinline__ void atomic_add_f32(float *p, float v) { unsafeAtomicAdd(p, v); }

// Wave-uniform node record through the scalar unit.
__device__ __forceinline__ Node load_node(const Node *p) {
    const uint2 raw = *reinterpret_cast<const uint2 *>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(raw.x), hi = __builtin_amdgcn_readfirstlane(raw.y);
    Node n;
    n.slot = (uint16_t)(lo & 0xFFFFu);
    n.hi = (uint16_t)(lo >> 16);
    n.lo = (uint16_t)(hi & 0xFFFFu);
    n.pad = 0;
    return n;
}

// z = sum_j q_j y_j - q0 in FP64 from the float32 y, multiply then add in stored order, no
// fused multiply-add: the exact atom test of the satisfaction check (and, at kappa = inf,
// of the hard objective) is bit-identical for every evaluator that follows this order.
__device__ __forceinline__ double atom_z_exact(const int32_t *ptr, const int32_t *var, const double *coef,
                                               const double *rhs, int k, const View &b, int r) {
#pragma clang fp contract(off)
    double acc = 0.0;
    const int e1 = ptr[k + 1];
    for (int e = ptr[k]; e < e1; ++e) {
        const double prod = coef[e] * (double)b.at(r, var[e]);
        acc = acc + prod;
    }
    return acc - rhs[k];
}

// Deterministic walk of constraint c's diagram at the rounded point of restart r.
__device__ __forceinline__ bool walk_exact(const TplInfo *tpl, const Node *nodes, const BucketInfo *bucket,
                                           const int32_t *con_bucket, const int32_t *con_local, const int32_t *sup,
                                           const int32_t *atom_ptr, const int32_t *atom_var, const double *atom_coef,
                                           const double *atom_rhs, const uint8_t *atom_strict, int n_bool,
                                           const View &a, const View &b, int c, int r) {
    const BucketInfo B = bucket[con_bucket[c]];
    const TplInfo T = tpl[B.tpl];
    const int32_t *s = sup + B.sup_base + con_local[c];
    const int N = T.n_nodes;
    int v = T.root;
    while (v < N) {
        const Node x = nodes[T.node_off + v];
        const int id = s[(int64_t)x.slot * B.n_pos];
        bool t;
        if (x.slot < T.n_bslots) {
            t = a.at(r, id) < 0.0f;
        } else {
            const int k = id - n_bool;
            const double z = atom_z_exact(atom_ptr, atom_var, atom_coef, atom_rhs, k, b, r);
            t = atom_strict[k] ? (z < 0.0) : (z <= 0.0);
        }
        v = t ? x.hi : x.lo;
    }
    return v == N;
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

fsmt_status fill_view(const fsmt_view &v, float value, hipStream_t st);
fsmt_status fill_f32(float *p, int64_t n, float value, hipStream_t st);
fsmt_status check_device_ptr(const void *p, int device, const char *name);
fsmt_status select_device(const fsmt_xbdd *h);

}  // namespace fsmt

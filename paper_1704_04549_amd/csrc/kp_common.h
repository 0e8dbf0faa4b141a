// Common definitions for the KSVD preconditioner library.
//
// The per-element numerical routines (elem_ops.h) are written once against a
// small "team" interface: a group of cooperating threads with a barrier and
// deterministic sum reductions.  On the GPU a team is one workgroup; the same
// source also builds for the host with a one-thread team, which the CPU test
// suite uses to check the arithmetic without a GPU.
#pragma once

#include <math.h>
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define KP_HD __host__ __device__
#define KP_DEV __device__
#define KP_INLINE __host__ __device__ inline
// always inlined on the device: no calls inside a kernel (the call ABI then
// handles the caller's registers)
#define KP_HD_FORCEINLINE __host__ __device__ __forceinline__
#else
#define KP_HD
#define KP_DEV
#define KP_INLINE inline
#define KP_HD_FORCEINLINE inline
#endif

namespace kp {

constexpr int kRecLen = 16;
constexpr int kMaxN = 32;

// ---------------------------------------------------------------- host team
struct HostTeam {
    int tid() const { return 0; }
    int size() const { return 1; }
    void sync() const {}
    // matrix-core Gram products: not on this team (see WaveTeam::gram16)
    template <class BF>
    bool gram16(const double*, int, int, BF, double*, double*) const { return false; }
    double sum(double v) const { return v; }
    double max(double v) const { return v; }
    // reduce k partial sums in place (v[0..k)); identity on one thread
    void sum_many(double* /*v*/, int /*k*/) const {}
    bool leader() const { return true; }
    // groups: independent sub-teams (one wave each on the GPU) that reduce
    // among themselves without a team barrier
    int groups() const { return 1; }
    int group() const { return 0; }
    int lane() const { return 0; }
    int group_size() const { return 1; }
    double group_sum(double v) const { return v; }
    // index of the largest |v[i*stride]| for i in [lo, hi) (lowest index on ties)
    int argmax_abs(const double* v, int stride, int lo, int hi) const {
        int best = lo;
        for (int i = lo + 1; i < hi; ++i)
            if (fabs(v[i * stride]) > fabs(v[best * stride])) best = i;
        return best;
    }
    // out[j] = sum_i Q[j*ldq + i] * v[i] for j < k
    void dots(const double* Q, long ldq, int k, const double* v, int len, double* out) const {
        for (int j = 0; j < k; ++j) {
            double s = 0.0;
            for (int i = 0; i < len; ++i) s += Q[j * ldq + i] * v[i];
            out[j] = s;
        }
    }
};

#if defined(__HIPCC__)
// ----------------------------------------------------------- workgroup team
// scratch: LDS array of at least (blockDim.x/64) * kMaxReduce doubles.
constexpr int kMaxReduce = 72;

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct BlockTeam {
    double* scratch;
    __device__ int tid() const { return (int)threadIdx.x; }
    __device__ int size() const { return (int)blockDim.x; }
    __device__ void sync() const { __syncthreads(); }
    template <class BF>
    __device__ bool gram16(const double*, int, int, BF, double*, double*) const { return false; }
    __device__ bool leader() const { return threadIdx.x == 0; }
    __device__ int groups() const { return (int)(blockDim.x >> 6); }
    __device__ int group() const { return (int)(threadIdx.x >> 6); }
    __device__ int lane() const { return (int)(threadIdx.x & 63); }
    __device__ int group_size() const { return 64; }
    __device__ double group_sum(double v) const { return wave_sum(v); }
    __device__ double sum(double v) const {
        const int nw = (int)(blockDim.x >> 6);
        v = wave_sum(v);
        if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
        __syncthreads();
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += scratch[w];
        __syncthreads();
        return s;
    }
    __device__ double max(double v) const {
        const int nw = (int)(blockDim.x >> 6);
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        if (nw == 1) return v;
        if ((threadIdx.x & 63) == 0) scratch[threadIdx.x >> 6] = v;
        __syncthreads();
        double m = scratch[0];
        for (int w = 1; w < nw; ++w) m = fmax(m, scratch[w]);
        __syncthreads();
        return m;
    }
    // index of the largest |v[i*stride]| for i in [lo, hi) (lowest index on ties);
    // every thread gets the answer
    __device__ int argmax_abs(const double* v, int stride, int lo, int hi) const {
        double bv = -1.0;
        int bi = lo;
        for (int i = lo + (int)threadIdx.x; i < hi; i += blockDim.x) {
            const double a = fabs(v[i * stride]);
            if (a > bv) { bv = a; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        const int nw = (int)(blockDim.x >> 6);
        if (nw == 1) return bi;
        if ((threadIdx.x & 63) == 0) {
            scratch[threadIdx.x >> 6] = bv;
            scratch[nw + (threadIdx.x >> 6)] = (double)bi;
        }
        __syncthreads();
        bv = scratch[0];
        bi = (int)scratch[nw];
        for (int w = 1; w < nw; ++w) {
            const double ov = scratch[w];
            const int oi = (int)scratch[nw + w];
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        __syncthreads();
        return bi;
    }
    // out[j] = sum_i Q[j*ldq + i] * v[i] for j < k; one wave per dot product,
    // fixed summation order; out is visible to the whole team on return.  A
    // wave forms 8 of its dot products at a time (their loads in flight
    // together, their reductions interleaved).
    __device__ void dots(const double* Q, long ldq, int k, const double* v, int len,
                         double* out) const {
        const int nw = (int)(blockDim.x >> 6);
        const int w = (int)(threadIdx.x >> 6), lane = (int)(threadIdx.x & 63);
        for (int j0 = w; j0 < k; j0 += 8 * nw) {
            double s[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] = 0.0;
            for (int i = lane; i < len; i += 64) {
                const double vi = v[i];
                // rows past k - 1 read row k - 1 (their sums are not stored):
                // the eight loads carry no condition, so none waits for another
                double qv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) qv[u] = Q[(long)min(j0 + u * nw, k - 1) * ldq + i];
#pragma unroll
                for (int u = 0; u < 8; ++u) s[u] += qv[u] * vi;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] = wave_sum(s[u]);
            if (lane == 0)
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + u * nw < k) out[j0 + u * nw] = s[u];
        }
        __syncthreads();
    }
    // v[0..k) hold per-thread partials on entry and the team sums on exit
    __device__ void sum_many(double* v, int k) const {
        const int nw = (int)(blockDim.x >> 6);
        const int w = (int)(threadIdx.x >> 6);
        for (int i = 0; i < k; ++i) {
            double t = wave_sum(v[i]);
            if ((threadIdx.x & 63) == 0) scratch[i * nw + w] = t;
        }
        __syncthreads();
        for (int i = 0; i < k; ++i) {
            double s = 0.0;
            for (int j = 0; j < nw; ++j) s += scratch[i * nw + j];
            v[i] = s;
        }
        __syncthreads();
    }
};

// ----------------------------------------------------------- wave team
// One wave (64 lanes) as a team of its own, independent of the other waves
// of its workgroup: sync is a wave-scope fence plus a wave barrier (no
// workgroup barrier), reductions are wave shuffles.  Routines that use only
// tid / size / sync / sum / max run unchanged on it.
// Sixteen lanes of a wave as a team: a wave runs four such teams on
// independent problems.  Control flow is uniform within a team (it may
// differ between the four); sync is the wave's fence, reductions stay within
// the team's lanes.
struct GroupTeam16 {
    __device__ int tid() const { return (int)(threadIdx.x & 15); }
    __device__ int size() const { return 16; }
    __device__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __device__ bool leader() const { return (threadIdx.x & 15) == 0; }
    __device__ double sum(double v) const {
        for (int off = 8; off > 0; off >>= 1) v += __shfl_xor(v, off, 16);
        return v;
    }
    __device__ double max(double v) const {
        for (int off = 8; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 16));
        return v;
    }
};

struct WaveTeam {
    __device__ int tid() const { return (int)(threadIdx.x & 63); }
    __device__ int size() const { return 64; }
    __device__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    // G = M M^T (rows x rows, row-major) and mv[j * rows + i] = (M V)[i][j]
    // for j = 0, 1, where M is rows x len row-major (rows <= 16, len a
    // multiple of 4) and V[q][j] = bf(q, j), on the FP64 matrix cores: per
    // 16x16x4 product the lane (g, c) loads M[c][q0 + g] once and feeds it as
    // both operands of M M^T.  G and mv are visible to the wave on return.
    // Returns false (nothing written) when the shape does not fit.
    template <class BF>
    __device__ bool gram16(const double* M, int rows, int len, BF bf, double* G, double* mv) const {
        if (rows > 16 || (len & 3)) return false;
        typedef double dx4 __attribute__((ext_vector_type(4)));
        const int lane = (int)(threadIdx.x & 63), g = lane >> 4, c = lane & 15;
        dx4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < len; q0 += 4) {
            const double a = c < rows ? M[(long)c * len + q0 + g] : 0.0;
            const double b = c < 2 ? bf(q0 + g, c) : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc2, 0, 0, 0);
        }
        // the lane holds D[g + 4 v][c]
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = g + 4 * v;
            if (r < rows && c < rows) G[r * rows + c] = acc[v];
            if (r < rows && c < 2) mv[c * rows + r] = acc2[v];
        }
        sync();
        return true;
    }
    __device__ bool leader() const { return (threadIdx.x & 63) == 0; }
    __device__ double sum(double v) const { return wave_sum(v); }
    __device__ double max(double v) const {
        for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
        return v;
    }
    // out[j] = sum_i Q[j*ldq + i] * v[i] for j < k (lanes over i, then the
    // wave reduction); out is visible to the wave on return.  Eight dot
    // products at a time: their loads in flight together, their reductions
    // interleaved (the summation order of each is unchanged).
    __device__ void dots(const double* Q, long ldq, int k, const double* v, int len, double* out) const {
        const int lane = (int)(threadIdx.x & 63);
        for (int j0 = 0; j0 < k; j0 += 8) {
            double s[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] = 0.0;
            for (int i = lane; i < len; i += 64) {
                const double vi = v[i];
                // rows past k - 1 read row k - 1 (their sums are not stored):
                // the eight loads carry no condition, so none waits for another
                double qv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) qv[u] = Q[(long)min(j0 + u, k - 1) * ldq + i];
#pragma unroll
                for (int u = 0; u < 8; ++u) s[u] += qv[u] * vi;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) s[u] = wave_sum(s[u]);
            if (lane == 0)
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + u < k) out[j0 + u] = s[u];
        }
        sync();
    }
    // v[0..k) hold per-lane partials on entry and the wave sums on exit
    __device__ void sum_many(double* v, int k) const {
        for (int i = 0; i < k; ++i) v[i] = wave_sum(v[i]);
    }
    // the wave is a single group
    __device__ int groups() const { return 1; }
    __device__ int group() const { return 0; }
    __device__ int lane() const { return (int)(threadIdx.x & 63); }
    __device__ int group_size() const { return 64; }
    __device__ double group_sum(double v) const { return wave_sum(v); }
    // index of the largest |v[i*stride]| for i in [lo, hi) (lowest index on ties)
    __device__ int argmax_abs(const double* v, int stride, int lo, int hi) const {
        double bv = -1.0;
        int bi = lo;
        for (int i = lo + (int)(threadIdx.x & 63); i < hi; i += 64) {
            const double a = fabs(v[i * stride]);
            if (a > bv) { bv = a; bi = i; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            const double ov = __shfl_xor(bv, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        return bi;
    }
};
#endif

// bf16 <-> f32 (round to nearest even), host and device.  The device form is
// the hardware converter (v_cvt_pk_bf16_f32, round to nearest even); the host
// form rounds the bit pattern.  They agree on every finite value (NaN
// payloads may differ).
KP_INLINE uint16_t f32_to_bf16(float f) {
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
#else
    union { float f; uint32_t u; } c;
    c.f = f;
    uint32_t u = c.u;
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
#endif
}
KP_INLINE float bf16_to_f32(uint16_t h) {
    union { float f; uint32_t u; } c;
    c.u = ((uint32_t)h) << 16;
    return c.f;
}

}  // namespace kp

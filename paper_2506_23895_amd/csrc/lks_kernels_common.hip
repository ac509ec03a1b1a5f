// Per-solve and per-reverse-step kernels shared by 2D and 3D:
//   design prep   kappa_ref = I(gamma), I'(gamma) on the design grid (Sec. 2.3, first equation)
//   init          X^0 with the composite boundary rules applied
//   sens gather   G(xi) += sum_x W_n(x - x_ref(xi)) kappa_bar^n(x): the transpose of the transfer
//                 as a gather onto each design node (one thread per design node, no atomics)
//   sens finish   dJ/dgamma = I'(gamma) G (Sec. 2.4, sensitivity pulled back to the design grid)
//   fill, non-finite scans (the whole state every few steps, recording the step of the first bad one)
#include "lks_device.hpp"

namespace lks {

template <typename T>
__global__ __launch_bounds__(kBlock) void k_design_prep(const T *gamma, T *kref, double *kprime,
                                                        long long nd, int interp, double kmax,
                                                        double q) {
    const long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
    if (i >= nd) return;
    const double g = (double)gamma[i];
    if (interp == 0) {  // gamma = 1 solid
        const double den = (1.0 - g) + q;
        kref[i] = (T)(kmax * q * g / den);
        kprime[i] = kmax * q * (1.0 + q) / (den * den);
    } else {            // gamma = 1 fluid
        const double den = q + g;
        kref[i] = (T)(kmax * q * (1.0 - g) / den);
        kprime[i] = -kmax * q * (1.0 + q) / (den * den);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_init(const InitArgs<T> a) {
    const Geom &g = a.g;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    const long long t = blockIdx.x * (long long)kBlock + threadIdx.x;
    if (t >= ncell) return;
    const unsigned tu = (unsigned)t, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];  // < 2^31 cells
    const int x = (int)(tu % n0), y = (int)((tu / n0) % n1), z = (int)(tu / (n0 * n1));
    if (on_face(g, 0, x) || on_face(g, 1, y) || (g.dim == 3 && on_face(g, 2, z))) return;
    const long long idx = x + y * g.sy + z * g.sz;
    T v[4];
    v[0] = a.rinit ? a.rinit[idx] : a.r0;
    for (int c = 0; c < 3; ++c) v[1 + c] = (c < g.dim) ? (a.uinit[0] ? a.uinit[c][idx] : a.u0[c]) : T(0);
    a.rout[idx] = v[0];
    for (int c = 0; c < g.dim; ++c) a.uout[c][idx] = v[1 + c];
    const int c3[3] = {x, y, z};
    push_boundary<T, 3>(g, a.bc, c3, v, [&](const int p[3], const T pv[4]) {
        const long long pi = p[0] + p[1] * g.sy + p[2] * g.sz;
        a.rout[pi] = pv[0];
        for (int c = 0; c < g.dim; ++c) a.uout[c][pi] = pv[1 + c];
    });
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sens_batch(const SensArgs<T> *__restrict__ args, const long long *__restrict__ blk0,
                                                       int njobs) {
    const long long b = blockIdx.x;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (blk0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    sens_body<T>(args[lo], njobs == 1 ? b : b - blk0[lo]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_sens_finish(const double *kprime, const double *G,
                                                        T *out, long long nd) {
    const long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
    if (i < nd) out[i] = (T)(kprime[i] * G[i]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill(T *p, T v, long long count) {
    const long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
    if (i < count) p[i] = v;
}

// Elements [0, np) of p then [0, nq) of q; a NaN/Inf records `step` in *flag: the smallest such
// step (keep_max = 0, forward sweep) or the largest (keep_max = 1, reverse sweep).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan(const T *p, long long np, const T *q, long long nq, int step,
                                                 int *flag, int keep_max) {
    const long long i = blockIdx.x * (long long)kBlock + threadIdx.x;
    bool bad = false;
    if (i < np) bad = !isfinite(p[i]);
    else if (i - np < nq) bad = !isfinite(q[i - np]);
    if (bad) {
        if (keep_max) atomicMax(flag, step);
        else atomicMin(flag, step);
    }
}

__global__ __launch_bounds__(kBlock) void k_reduce_steps(const double *partials, long long stride,
                                                         long long nblocks, int n0, double scale,
                                                         double *jn) {
    __shared__ double sh4[4];
    const int n = n0 + blockIdx.x;
    const double *row = partials + (long long)blockIdx.x * stride;
    double acc = 0.0;
    for (long long i = threadIdx.x; i < nblocks; i += kBlock) acc += row[i];
    const double t = block_sum(acc, sh4);
    if (threadIdx.x == 0) jn[n] = t * scale;
}

static inline dim3 grid1(long long n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

template <typename T>
hipError_t launch_design_prep(const T *gamma, T *kref, double *kprime, long long nd, int interp,
                              double kmax, double q, hipStream_t s) {
    hipLaunchKernelGGL(k_design_prep<T>, grid1(nd), dim3(kBlock), 0, s, gamma, kref, kprime, nd,
                       interp, kmax, q);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init(const InitArgs<T> &a, hipStream_t s) {
    const long long ncell = (long long)a.g.n[0] * a.g.n[1] * a.g.n[2];
    hipLaunchKernelGGL(k_init<T>, grid1(ncell), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sens_batch(const SensArgs<T> *args, const long long *blk0, int njobs, long long nblk,
                             hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sens_batch<T>, dim3((unsigned)nblk), dim3(kBlock), 0, s, args, blk0, njobs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sens_finish(const double *kprime, const double *G, T *out, long long nd,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_sens_finish<T>, grid1(nd), dim3(kBlock), 0, s, kprime, G, out, nd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *p, T v, long long count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<T>, grid1(count), dim3(kBlock), 0, s, p, v, count);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scan(const T *p, long long np, const T *q, long long nq, int step, int *flag, int keep_max,
                       hipStream_t s) {
    if (np + nq <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan<T>, grid1(np + nq), dim3(kBlock), 0, s, p, np, q, nq, step, flag, keep_max);
    return hipGetLastError();
}

hipError_t launch_reduce_steps(const double *partials, long long stride, long long nblocks, int n0,
                               int n1, double scale, double *jn, hipStream_t s) {
    if (n1 < n0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_steps, dim3(n1 - n0 + 1), dim3(kBlock), 0, s, partials, stride,
                       nblocks, n0, scale, jn);
    return hipGetLastError();
}

#define LKS_INST(T)                                                                               \
    template hipError_t launch_design_prep<T>(const T *, T *, double *, long long, int, double,   \
                                              double, hipStream_t);                               \
    template hipError_t launch_init<T>(const InitArgs<T> &, hipStream_t);                         \
    template hipError_t launch_sens_batch<T>(const SensArgs<T> *, const long long *, int, long long, \
                                             hipStream_t);                                        \
    template hipError_t launch_sens_finish<T>(const double *, const double *, T *, long long,     \
                                              hipStream_t);                                       \
    template hipError_t launch_fill<T>(T *, T, long long, hipStream_t);                           \
    template hipError_t launch_scan<T>(const T *, long long, const T *, long long, int, int *, int, \
                                       hipStream_t);
LKS_INST(float)
LKS_INST(double)
template hipError_t launch_fill<unsigned int>(unsigned int *, unsigned int, long long, hipStream_t);
template hipError_t launch_fill<int>(int *, int, long long, hipStream_t);
#undef LKS_INST

}  // namespace lks

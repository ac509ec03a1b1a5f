// Device helpers shared by the 2D and 3D kernels: the transfer gather (design -> analysis), the
// composite boundary rules, the objective densities and deterministic block reductions.
#pragma once

#include "lks_internal.hpp"

namespace lks {

enum { BC_PERIODIC = 0, BC_VELOCITY = 1, BC_PRESSURE = 2, BC_ZERO_GRADIENT = 3, BC_NOSLIP = 4 };
enum { OBJ_NONE = -1, OBJ_POWER = 0, OBJ_DRAG = 1, OBJ_TORQUE = 2, OBJ_J1 = 3, OBJ_J2 = 4,
       OBJ_MASS = 5 };

constexpr int kBlock = 256;

// Pointers read out of an argument block are generic (flat) to the compiler, and flat loads count
// against both the vector-memory and the LDS/scalar wait counters: every LDS or scalar wait would
// then also drain all outstanding field loads.  Field accesses go through these casts to the global
// address space, so they count against the vector-memory counter only.
#define LKS_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const LKS_GLOBAL T *gld(const T *p) { return (const LKS_GLOBAL T *)p; }
template <typename T>
__device__ __forceinline__ LKS_GLOBAL T *gst(T *p) { return (LKS_GLOBAL T *)p; }

// Argument blocks are read through the scalar cache field by field as the code reaches them, so
// each 64-byte line first read behind a branch costs one more memory round trip before a wave's
// first field load.  Touching every line of the block at once puts those misses in one round trip
// (2D forward at 1024^2: 11.5 -> 10.9 us per launch).  The 3D kernels do not take it: their
// blocks march for hundreds of microseconds, and the 3D forward measured slower with it.
#define LKS_CONST __attribute__((address_space(4)))
template <int BYTES>
__device__ __forceinline__ void touch_lines(const void *p) {
    const LKS_CONST unsigned *q = (const LKS_CONST unsigned *)p;
    unsigned acc = q[BYTES / 4 - 1];
#pragma unroll
    for (int o = 0; o < BYTES / 4; o += 16) acc |= q[o];
    asm volatile("" ::"r"(acc));  // keeps the loads (emits no instruction)
}

// At the end of its work, one wave per XCD (blocks are dealt to the eight XCDs in turn) touches
// the argument block of the next launch on the stream, so that launch finds it in cache instead
// of in HBM (2D forward at 1024^2: 10.9 -> 10.6 us per launch).
template <int BYTES>
__device__ __forceinline__ void prefetch_next(const void *next) {
    if (next && blockIdx.x < 8 && threadIdx.x < 64) touch_lines<BYTES>(next);
}

// ---- lane shifts within a 64-wide wavefront (DPP wave_shr:1 / wave_shl:1; edge lanes read 0) ----
__device__ __forceinline__ int dpp_l(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_r(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, true); }
// value of lane i-1 / lane i+1
__device__ __forceinline__ float from_left(float v) { return __builtin_bit_cast(float, dpp_l(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ float from_right(float v) { return __builtin_bit_cast(float, dpp_r(__builtin_bit_cast(int, v))); }
__device__ __forceinline__ double from_left(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_l((int)(b & 0xffffffffLL)), hi = dpp_l((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_right(double v) {
    const long long b = __builtin_bit_cast(long long, v);
    const int lo = dpp_r((int)(b & 0xffffffffLL)), hi = dpp_r((int)(b >> 32));
    return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// wrap a coordinate onto a periodic axis; false if it leaves a non-periodic axis
__device__ __forceinline__ bool wrapc(int &v, int n, int per) {
    if (v >= 0 && v < n) return true;
    if (!per) return false;
    v %= n;
    if (v < 0) v += n;
    return true;
}

__device__ __forceinline__ bool on_face(const Geom &g, int a, int c) {
    return !g.per[a] && (c == 0 || c == g.n[a] - 1);
}

// cos(pi v / 2) for |v| < 2: the hardware cosine in single precision, cospi in double
__device__ __forceinline__ float cos_half_pi(float v) { return __cosf(v * 1.57079632679489662f); }
__device__ __forceinline__ double cos_half_pi(double v) { return cospi(v * 0.5); }

// Transfer weight w(r) (Sec. 2.3 weight functions): LIN hat, or Peskin's cosine (1 + cos) / 4.
template <typename T>
__device__ __forceinline__ T wk(int weight, T d) {
    T a = fabs(d);
    if (weight == 1) return a < T(1) ? T(1) - a : T(0);
    return a < T(2) ? T(0.25) * (T(1) + cos_half_pi(d)) : T(0);
}

// kappa(x) = sum_xi W(x - x_ref(xi)) kappa_ref(xi) and u_S(x) = sum_xi W u_ref(xi) at one analysis
// node (Eqs. brinkman_ref, velocity_ref), evaluated as a gather: x is mapped back into the
// design frame, p = R^T (x - xG) + xi_G, and the design nodes whose image can lie within the
// kernel support of x are scanned.  x - x_ref(xi) = R (p - xi); u_ref is affine in xi, so
// sum W u_ref = Omega x ((x - xG) sum W - sum W (x - x_ref)) + uG sum W.
template <typename T, int DIM>
__device__ __forceinline__ void gather_kappa(const Design<T> &des, const StepMotion &m, int x, int y,
                                             int z, T &kap, T us[3]) {
    constexpr int dim = DIM;
    const double dx = x - m.xG[0], dy = y - m.xG[1], dz = (dim == 3) ? z - m.xG[2] : 0.0;
    double p[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) p[b] = m.R[b] * dx + m.R[3 + b] * dy + m.R[6 + b] * dz + des.xiG[b];
    const double s = des.weight == 1 ? 1.0 : 2.0;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int b = 0; b < dim; ++b) {
        double h = 0.0;
#pragma unroll
        for (int a = 0; a < dim; ++a) h += fabs(m.R[3 * a + b]);
        h *= s;
        lo[b] = max(0, (int)ceil(p[b] - h));
        hi[b] = min(des.nd[b] - 1, (int)floor(p[b] + h));
    }
    T R[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = (T)m.R[i];
    T f[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int b = 0; b < dim; ++b) f[b] = (T)(p[b] - lo[b]);
    T d0[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) d0[a] = R[3 * a] * f[0] + R[3 * a + 1] * f[1] + R[3 * a + 2] * f[2];
    // along a candidate row (fixed j, k) d_a is affine in fi: d_a = c_a - fi R[3a]; the nodes
    // with |d_a| < s on every axis form one interval of fi, so only that interval is scanned
    // (slightly widened against rounding: nodes outside the support still get W = 0 below)
    const T sT = (T)s, span = (T)(hi[0] - lo[0]);
    T inv[3];
#pragma unroll
    for (int a = 0; a < dim; ++a) inv[a] = fabs(R[3 * a]) > T(1e-6) ? T(1) / R[3 * a] : T(0);
    T sW = 0, sWk = 0, sWd[3] = {0, 0, 0};
    if (DIM == 3 && m.R[2] == 0.0 && m.R[5] == 0.0 && m.R[6] == 0.0 && m.R[7] == 0.0 &&
        m.R[8] == 1.0) {
        // Rotation about z (the same for the whole launch): d_z depends on the plane alone and
        // the x/y window is the same on every plane, so the x/y weights are formed once per
        // (i, j) and the planes of the support (at most 2s + 1 <= 5) are summed innermost.
        constexpr int MK = 5;
        const int nk = hi[2] - lo[2] + 1;
        T wz[MK], dz[MK];
#pragma unroll
        for (int kk = 0; kk < MK; ++kk) {
            dz[kk] = d0[2] - (T)kk;
            wz[kk] = kk < nk ? wk<T>(des.weight, dz[kk]) : T(0);
        }
        const long long pst = (long long)des.nd[0] * des.nd[1];
        const int kl = max(nk - 1, 0);
        for (int j = lo[1]; j <= hi[1] && nk > 0; ++j) {
            const T fj = (T)(j - lo[1]);
            T flo = T(0), fhi = span;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const T ca = d0[a] - fj * R[3 * a + 1];
                if (inv[a] != T(0)) {
                    const T t1 = (ca - sT) * inv[a], t2 = (ca + sT) * inv[a];
                    flo = fmax(flo, fmin(t1, t2) - T(1e-3));
                    fhi = fmin(fhi, fmax(t1, t2) + T(1e-3));
                } else if (fabs(ca) >= sT + T(1e-3)) {
                    fhi = T(-1);
                }
            }
            if (flo > fhi) continue;
            const int i0 = lo[0] + (int)ceil(flo), i1 = lo[0] + (int)floor(fhi);
            const T *krow = des.kref + (long long)des.nd[0] * (j + (long long)des.nd[1] * lo[2]);
            for (int i = i0; i <= i1; ++i) {
                const T fi = (T)(i - lo[0]);
                const T dx = d0[0] - fi * R[0] - fj * R[1], dy = d0[1] - fi * R[3] - fj * R[4];
                const T wxy = wk<T>(des.weight, dx) * wk<T>(des.weight, dy);
                if (wxy == T(0)) continue;
                // planes beyond the support read the last one (a valid node) with weight zero
                T kv[MK];
#pragma unroll
                for (int kk = 0; kk < MK; ++kk) kv[kk] = krow[i + min(kk, kl) * pst];
#pragma unroll
                for (int kk = 0; kk < MK; ++kk) {
                    const T W = wxy * wz[kk];
                    sW += W;
                    sWk += W * kv[kk];
                    sWd[0] += W * dx;
                    sWd[1] += W * dy;
                    sWd[2] += W * dz[kk];
                }
            }
        }
    } else
    for (int k = lo[2]; k <= hi[2]; ++k) {
        const T fk = (T)(k - lo[2]);
        for (int j = lo[1]; j <= hi[1]; ++j) {
            const T fj = (T)(j - lo[1]);
            T flo = T(0), fhi = span;
#pragma unroll
            for (int a = 0; a < dim; ++a) {
                const T ca = d0[a] - fj * R[3 * a + 1] - fk * R[3 * a + 2];
                if (inv[a] != T(0)) {
                    const T t1 = (ca - sT) * inv[a], t2 = (ca + sT) * inv[a];
                    flo = fmax(flo, fmin(t1, t2) - T(1e-3));
                    fhi = fmin(fhi, fmax(t1, t2) + T(1e-3));
                } else if (fabs(ca) >= sT + T(1e-3)) {
                    fhi = T(-1);
                }
            }
            if (flo > fhi) continue;
            const int i0 = lo[0] + (int)ceil(flo), i1 = lo[0] + (int)floor(fhi);
            const T *krow = des.kref + (long long)des.nd[0] * (j + (long long)des.nd[1] * k);
            for (int i = i0; i <= i1; i += 4) {  // four candidates' loads in flight together
                T kv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) kv[u] = i + u <= i1 ? krow[i + u] : T(0);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (i + u > i1) break;
                    const T fi = (T)(i + u - lo[0]);
                    T d[3] = {T(0), T(0), T(0)}, W = T(1);
#pragma unroll
                    for (int a = 0; a < dim; ++a) {
                        d[a] = d0[a] - fi * R[3 * a] - fj * R[3 * a + 1] - fk * R[3 * a + 2];
                        W *= wk<T>(des.weight, d[a]);
                    }
                    if (W == T(0)) continue;
                    sW += W;
                    sWk += W * kv[u];
#pragma unroll
                    for (int a = 0; a < dim; ++a) sWd[a] += W * d[a];
                }
            }
        }
    }
    kap = sWk;
    const double r0 = dx * (double)sW - (double)sWd[0];
    const double r1 = dy * (double)sW - (double)sWd[1];
    const double r2 = dz * (double)sW - (double)sWd[2];
    us[0] = (T)(m.Om[1] * r2 - m.Om[2] * r1 + m.uG[0] * (double)sW);
    us[1] = (T)(m.Om[2] * r0 - m.Om[0] * r2 + m.uG[1] * (double)sW);
    us[2] = dim == 3 ? (T)(m.Om[0] * r1 - m.Om[1] * r0 + m.uG[2] * (double)sW) : T(0);
}

__device__ __forceinline__ bool in_box(const StepMotion &m, int dim, int x, int y, int z) {
    bool in = x >= m.lo[0] && x <= m.hi[0] && y >= m.lo[1] && y <= m.hi[1];
    if (dim == 3) in = in && z >= m.lo[2] && z <= m.hi[2];
    return in;
}

__device__ __forceinline__ long long box_index(const BoxGeom &b, const StepMotion &m, int dim,
                                               int x, int y, int z) {
    return (x - m.lo[0]) + (long long)(y - m.lo[1]) * b.bsy +
           (dim == 3 ? (long long)(z - m.lo[2]) * b.bsz : 0LL);
}

// 2D box index of (x, y) clamped into the step's box: always a valid element, so a load from it
// needs no per-lane branch (the caller selects zero where the node is outside).  Boxes hold fewer
// than 2^31 nodes, so 32-bit arithmetic suffices.
__device__ __forceinline__ int box_index2_clamped(const BoxGeom &b, const StepMotion &m, int x, int y) {
    const int cx = min(max(x, m.lo[0]), m.hi[0]), cy = min(max(y, m.lo[1]), m.hi[1]);
    return (cx - m.lo[0]) + (cy - m.lo[1]) * (int)b.bsy;
}

// Transfer of one step onto its footprint box, one thread per box cell: writes kappa and u_S
// into box arrays (fixed extent bn, this step's origin m.lo).  Launched as extra blocks of the
// previous step's stencil launch, so it runs off the stencil's critical path.
template <typename T, int DIM, int NT>
__device__ __forceinline__ void transfer_box(const Design<T> &des, const StepMotion &m,
                                             const BoxGeom &box, T *kout, T *const usout[3],
                                             long long blk) {
    const long long cell = blk * NT + threadIdx.x;
    const int ex = m.hi[0] - m.lo[0] + 1, ey = m.hi[1] - m.lo[1] + 1;
    const int ez = DIM == 3 ? m.hi[2] - m.lo[2] + 1 : 1;
    if (cell >= (long long)ex * ey * ez) return;
    // 32-bit division: box extents are validated below 2^31 cells at create
    const unsigned cu = (unsigned)cell, uex = (unsigned)ex, uey = (unsigned)ey;
    const int bx = (int)(cu % uex), by = (int)((cu / uex) % uey), bz = (int)(cu / (uex * uey));
    T kap, us[3];
    gather_kappa<T, DIM>(des, m, m.lo[0] + bx, m.lo[1] + by, DIM == 3 ? m.lo[2] + bz : 0, kap, us);
    const long long bi = bx + by * box.bsy + (DIM == 3 ? bz * box.bsz : 0LL);
    kout[bi] = kap;
#pragma unroll
    for (int a = 0; a < DIM; ++a) usout[a][bi] = us[a];
}

// ---- composite boundary rules ------------------------------------------------------------
// Faces are applied in the order x-, x+, y-, y+, z-, z+ and each face rule reads the next node
// inward, which is already final when that face is applied.  So a face node p takes its value
// from exactly one interior node s (p shifted inward along each face it lies on), and each
// component either survives every face of p's chain (copied from s) or is fixed by the latest
// face of the chain that prescribes it.  comp 0 = rho, comp 1 + b = u_b.
__device__ __forceinline__ bool bc_copies(int kind, int comp, int axis) {
    if (comp == 0) return kind == BC_VELOCITY || kind == BC_NOSLIP;
    return kind == BC_ZERO_GRADIENT || (kind == BC_PRESSURE && comp - 1 == axis);
}

template <typename T>
__device__ __forceinline__ T bc_const(const BCParams<T> &bc, int f, int comp) {
    return comp == 0 ? bc.rho[f] : bc.u[f][comp - 1];
}

// side[a] = 0 if interior node c is next to face a-, 1 if next to a+, -1 otherwise; returns the
// bit set of adjacent axes
template <int DIM>
__device__ __forceinline__ int adjacent_faces(const Geom &g, const int c[3], int side[3]) {
    int bits = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        side[a] = -1;
        if (a >= DIM || g.per[a]) continue;
        if (c[a] == 1) side[a] = 0;
        else if (c[a] == g.n[a] - 2) side[a] = 1;
        if (side[a] >= 0) bits |= 1 << a;
    }
    return bits;
}

// Forward: write every face node whose chain ends at interior node c (value v[0..dim]).  The face
// nodes are c shifted outward along each non-empty subset of the adjacent axes.
template <typename T, int DIM, typename Emit>
__device__ void push_boundary(const Geom &g, const BCParams<T> &bc, const int c[3], const T v[4],
                              Emit &&emit) {
    int side[3];
    const int bits = adjacent_faces<DIM>(g, c, side);
    if (bits == 0) return;
    for (int mask = 1; mask < (1 << DIM); ++mask) {
        if ((mask & bits) != mask) continue;
        int p[3] = {c[0], c[1], c[2]};
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            if ((mask >> a) & 1) p[a] = side[a] ? g.n[a] - 1 : 0;
        T pv[4] = {v[0], v[1], v[2], v[3]};
#pragma unroll
        for (int comp = 0; comp <= DIM; ++comp) {
            bool done = false;
#pragma unroll
            for (int a = DIM - 1; a >= 0; --a) {  // latest face of the chain first
                if (done || !((mask >> a) & 1)) continue;
                const int f = 2 * a + side[a];
                if (!bc_copies(bc.kind[f], comp, a)) {
                    pv[comp] = bc_const(bc, f, comp);
                    done = true;
                }
            }
        }
        emit(p, pv);
    }
}

// Reverse: the seeds that face nodes pass back to interior node c.  fetch(p, comp) returns the
// seed of component comp at face node p; a component passes only if every face of the chain
// copies it.  Adds into acc[0..dim].
template <int DIM, typename Fetch, typename T>
__device__ void gather_boundary_T(const Geom &g, const int kind[6], const int c[3], T acc[4],
                                  Fetch &&fetch) {
    int side[3];
    const int bits = adjacent_faces<DIM>(g, c, side);
    if (bits == 0) return;
    for (int mask = 1; mask < (1 << DIM); ++mask) {
        if ((mask & bits) != mask) continue;
        int p[3] = {c[0], c[1], c[2]};
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            if ((mask >> a) & 1) p[a] = side[a] ? g.n[a] - 1 : 0;
#pragma unroll
        for (int comp = 0; comp <= DIM; ++comp) {
            bool pass = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                if ((mask >> a) & 1) pass = pass && bc_copies(kind[2 * a + side[a]], comp, a);
            if (pass) acc[comp] += fetch(p, comp);
        }
    }
}

// ---- objective density and its partials (per node, unscaled, mask applied by the caller) --
template <typename T>
__device__ __forceinline__ double obj_density(const ObjParams &o, int x, int y, int z, double r,
                                              const T u[3], T kap, const T us[3]) {
    const double F0 = (double)kap * ((double)u[0] - (double)us[0]);
    const double F1 = (double)kap * ((double)u[1] - (double)us[1]);
    const double F2 = (double)kap * ((double)u[2] - (double)us[2]);
    switch (o.kind) {
    case OBJ_DRAG: return F0 * o.dir[0] + F1 * o.dir[1] + F2 * o.dir[2];
    case OBJ_POWER: return F0 * (double)us[0] + F1 * (double)us[1] + F2 * (double)us[2];
    case OBJ_TORQUE: {
        const double r0 = x - o.centre[0], r1 = y - o.centre[1], r2 = z - o.centre[2];
        return o.dir[0] * (r1 * F2 - r2 * F1) + o.dir[1] * (r2 * F0 - r0 * F2) +
               o.dir[2] * (r0 * F1 - r1 * F0);
    }
    case OBJ_J1: return -(1.0 + r) / 3.0;  // r is rho - 1
    case OBJ_J2: return -(o.dir[0] * (double)u[0] + o.dir[1] * (double)u[1] + o.dir[2] * (double)u[2]);
    case OBJ_MASS: return 1.0 + r;
    }
    return 0.0;
}

// d(density)/d(rho, u) -> dP, dV[3]; d/d kappa needs u and is returned by obj_dkappa
__device__ __forceinline__ void obj_dstate(const ObjParams &o, int x, int y, int z, double kap,
                                           const double us[3], double &dP, double dV[3]) {
    dP = 0.0;
    dV[0] = dV[1] = dV[2] = 0.0;
    switch (o.kind) {
    case OBJ_DRAG:
        for (int a = 0; a < 3; ++a) dV[a] = kap * o.dir[a];
        break;
    case OBJ_POWER:
        for (int a = 0; a < 3; ++a) dV[a] = kap * us[a];
        break;
    case OBJ_TORQUE: {
        const double r0 = x - o.centre[0], r1 = y - o.centre[1], r2 = z - o.centre[2];
        dV[0] = kap * (o.dir[1] * r2 - o.dir[2] * r1);
        dV[1] = kap * (o.dir[2] * r0 - o.dir[0] * r2);
        dV[2] = kap * (o.dir[0] * r1 - o.dir[1] * r0);
        break;
    }
    case OBJ_J1: dP = -1.0 / 3.0; break;
    case OBJ_J2:
        for (int a = 0; a < 3; ++a) dV[a] = -o.dir[a];
        break;
    case OBJ_MASS: dP = 1.0; break;
    }
}

__device__ __forceinline__ double obj_dkappa(const ObjParams &o, int x, int y, int z,
                                             const double u[3], const double us[3]) {
    const double v0 = u[0] - us[0], v1 = u[1] - us[1], v2 = u[2] - us[2];
    switch (o.kind) {
    case OBJ_DRAG: return v0 * o.dir[0] + v1 * o.dir[1] + v2 * o.dir[2];
    case OBJ_POWER: return v0 * us[0] + v1 * us[1] + v2 * us[2];
    case OBJ_TORQUE: {
        const double r0 = x - o.centre[0], r1 = y - o.centre[1], r2 = z - o.centre[2];
        const double m0 = o.dir[1] * r2 - o.dir[2] * r1, m1 = o.dir[2] * r0 - o.dir[0] * r2,
                     m2 = o.dir[0] * r1 - o.dir[1] * r0;
        return v0 * m0 + v1 * m1 + v2 * m2;
    }
    }
    return 0.0;
}

// The same two partials in the arithmetic type R of the caller (R = double reproduces the two
// functions above operation for operation).
template <typename R>
__device__ __forceinline__ void obj_dstate_r(const ObjParams &o, int x, int y, int z, R kap, const R us[3],
                                             R &dP, R dV[3]) {
    dP = R(0);
    dV[0] = dV[1] = dV[2] = R(0);
    switch (o.kind) {
    case OBJ_DRAG:
        for (int a = 0; a < 3; ++a) dV[a] = kap * (R)o.dir[a];
        break;
    case OBJ_POWER:
        for (int a = 0; a < 3; ++a) dV[a] = kap * us[a];
        break;
    case OBJ_TORQUE: {
        const R r0 = (R)(x - o.centre[0]), r1 = (R)(y - o.centre[1]), r2 = (R)(z - o.centre[2]);
        dV[0] = kap * ((R)o.dir[1] * r2 - (R)o.dir[2] * r1);
        dV[1] = kap * ((R)o.dir[2] * r0 - (R)o.dir[0] * r2);
        dV[2] = kap * ((R)o.dir[0] * r1 - (R)o.dir[1] * r0);
        break;
    }
    case OBJ_J1: dP = R(-1.0 / 3.0); break;
    case OBJ_J2:
        for (int a = 0; a < 3; ++a) dV[a] = -(R)o.dir[a];
        break;
    case OBJ_MASS: dP = R(1); break;
    }
}

template <typename R>
__device__ __forceinline__ R obj_dkappa_r(const ObjParams &o, int x, int y, int z, const R u[3], const R us[3]) {
    const R v0 = u[0] - us[0], v1 = u[1] - us[1], v2 = u[2] - us[2];
    switch (o.kind) {
    case OBJ_DRAG: return v0 * (R)o.dir[0] + v1 * (R)o.dir[1] + v2 * (R)o.dir[2];
    case OBJ_POWER: return v0 * us[0] + v1 * us[1] + v2 * us[2];
    case OBJ_TORQUE: {
        const R r0 = (R)(x - o.centre[0]), r1 = (R)(y - o.centre[1]), r2 = (R)(z - o.centre[2]);
        const R m0 = (R)o.dir[1] * r2 - (R)o.dir[2] * r1, m1 = (R)o.dir[2] * r0 - (R)o.dir[0] * r2,
                m2 = (R)o.dir[0] * r1 - (R)o.dir[1] * r0;
        return v0 * m0 + v1 * m1 + v2 * m2;
    }
    }
    return R(0);
}

__device__ __forceinline__ bool obj_uses_kappa(int kind) {
    return kind == OBJ_DRAG || kind == OBJ_POWER || kind == OBJ_TORQUE;
}

// ---- deterministic reductions ---------------------------------------------------------------
// Sum over a block of NT threads in a fixed order; the result is valid on thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_t(double v, double *sh) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) t += sh[i];
    return t;
}

__device__ __forceinline__ double block_sum(double v, double *sh4) { return block_sum_t<256>(v, sh4); }

// Every block stores its partial for this step; the partials of all steps are summed in block
// order by one reduction kernel at the end of the sweep (no cross-block synchronisation here).
template <int NT = 256>
__device__ __forceinline__ void store_partial(const ObjParams &o, double v, long long blin,
                                              double *sh) {
    const double bs = block_sum_t<NT>(v, sh);
    if (threadIdx.x == 0) o.partials[blin] = bs;
}

// Blocks of a launch are dispatched round-robin over the 8 XCDs, each with its own L2.  Tile of
// the t-th dispatched block out of T: XCD t % 8 gets a contiguous run of tiles (row-major), so
// row chunks that share halo rows run on the same XCD close in time and the halos hit its L2.
// Odd XCDs walk their run backwards, so the last run (the bottom face rows, slower code) starts
// early instead of forming the tail of the launch.
__device__ __forceinline__ long long xcd_tile(long long t, long long T) {
    const long long q = T >> 3, r = T & 7, x = t & 7, l = t >> 3;
    const long long n = q + (x < r ? 1 : 0);
    return x * q + (x < r ? x : r) + ((x & 1) ? n - 1 - l : l);
}

// ---- sensitivity gather (one thread per design node) ------------------------------------------
// G(xi) += sum_x W(x - x_ref(xi)) kappa_bar(x) over the step's footprint box: the weight is a
// product over analysis axes and the support spans at most 2s + 1 nodes per axis, so per-axis
// weights are formed first and every load of a z-plane is issued together.
// Taps of an MW x MW window per z-plane: the weight is a product over analysis axes, so per-axis
// weights are formed first.  The window's origin is clamped into the step's box and the kappa_bar
// allocation is padded by 4 box rows + 8 nodes, so every tap address is in bounds and every load
// of a plane is issued unconditionally (one 64-bit address per row, columns as immediate offsets);
// taps outside [lo, hi] have weight 0 and are dropped by selection, never multiplied.
template <typename T, int MW>
__device__ __forceinline__ double sens_window(const SensArgs<T> &a, const int lo[3], const int hi[3],
                                              const double xr[3]) {
    T wx[MW], wy[MW];
#pragma unroll
    for (int t = 0; t < MW; ++t) {
        wx[t] = lo[0] + t <= hi[0] ? wk<T>(a.des.weight, (T)(lo[0] + t - xr[0])) : T(0);
        wy[t] = lo[1] + t <= hi[1] ? wk<T>(a.des.weight, (T)(lo[1] + t - xr[1])) : T(0);
    }
    const LKS_GLOBAL T *__restrict__ kb = gld(a.kbar);
    const int ox = min(lo[0], a.m.hi[0]), oy = min(lo[1], a.m.hi[1]);
    const long long bsy = a.box.bsy;
    double acc = 0.0;
    for (int z = lo[2]; z <= hi[2]; ++z) {
        const T wz = (a.dim == 3) ? wk<T>(a.des.weight, (T)(z - xr[2])) : T(1);
        if (wz == T(0)) continue;
        const LKS_GLOBAL T *r0 = kb + box_index(a.box, a.m, a.dim, ox, oy, z);
        T kv[MW][MW];
#pragma unroll
        for (int ty = 0; ty < MW; ++ty)
#pragma unroll
            for (int tx = 0; tx < MW; ++tx) kv[ty][tx] = r0[ty * bsy + tx];
#pragma unroll
        for (int ty = 0; ty < MW; ++ty)
#pragma unroll
            for (int tx = 0; tx < MW; ++tx)
                if (wx[tx] != T(0) && wy[ty] != T(0))
                    acc += (double)(wx[tx] * wy[ty] * wz) * (double)kv[ty][tx];
    }
    return acc;
}

template <typename T>
__device__ __forceinline__ void sens_body(const SensArgs<T> &a, long long blk) {
    const long long ndn = (long long)a.des.nd[0] * a.des.nd[1] * a.des.nd[2];
    const long long i = blk * kBlock + threadIdx.x;
    if (i >= ndn) return;
    const unsigned iu = (unsigned)i, n0 = (unsigned)a.des.nd[0], n1 = (unsigned)a.des.nd[1];
    const int ix = (int)(iu % n0), iy = (int)((iu / n0) % n1), iz = (int)(iu / (n0 * n1));  // < 2^31
    const double d0 = ix - a.des.xiG[0], d1 = iy - a.des.xiG[1],
                 d2 = (a.dim == 3) ? iz - a.des.xiG[2] : 0.0;
    double xr[3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
        xr[r] = a.m.R[3 * r] * d0 + a.m.R[3 * r + 1] * d1 + a.m.R[3 * r + 2] * d2 + a.m.xG[r];
    const double s = a.des.weight == 1 ? 1.0 : 2.0;
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int r = 0; r < a.dim; ++r) {
        lo[r] = max(a.m.lo[r], (int)ceil(xr[r] - s));
        hi[r] = min(a.m.hi[r], (int)floor(xr[r] + s));
    }
    // LIN support: at most 3 nodes per axis; COS4: at most 5 (weight kind is uniform per job)
    const double acc = a.des.weight == 1 ? sens_window<T, 3>(a, lo, hi, xr) : sens_window<T, 5>(a, lo, hi, xr);
    a.G[i] += acc;
}

}  // namespace lks

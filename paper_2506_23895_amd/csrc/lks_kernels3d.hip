// 3D kernels (D3Q19 and D3Q15).
//
// Forward step, marching along z (Algorithm 1 body, Sec. 2.2-2.3): a block owns a TX x TY column
// of output nodes and a chunk of zc planes (chosen per grid, 8..32, by choose_zc3).  Velocity
// planes z-2 .. z+2 (x-y halo 2) sit in an LDS ring; the equilibrium E_i of plane z (x-y halo 1)
// is evaluated once into LDS; each thread then adds the E_i pulled by its own column into three
// in-flight output planes held in registers (c_z = -1 completes plane z-1, c_z = 0 feeds plane z,
// c_z = +1 plane z+1), and finishes plane z-1: transfer gather, VPM update, composite boundary
// rules, objective partial.
// The next velocity plane is fetched into registers before the stencil work of the current one.
//
// Adjoint step in two kernels.  The first is pointwise: lambda = Lambda^n + dj^n/dX^n, the
// boundary transpose (seeds of face nodes returned to the interior node they copy from), the
// force transpose V* = V / (1 + kappa + kappa_s) and kappa_bar on the footprint box.  The second
// marches along z: (P*, V*) planes (halo 3) in an LDS ring, the pull transpose and its w-weighted
// moments rho~, u~, s~ per plane (halo 2; a ring of five s~ planes), and Lambda^{n-1} of the
// plane two behind from the transposed equilibrium and the transposed strain operator.
#include <type_traits>

#include "lks_device.hpp"

namespace lks {

// ---- velocity sets ----------------------------------------------------------------------------
template <int Q>
__device__ constexpr int cq(int i, int a);

template <>
__device__ constexpr int cq<19>(int i, int a) {
    constexpr int t[19][3] = {{0, 0, 0},  {1, 0, 0},   {-1, 0, 0}, {0, 1, 0},  {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1},  {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                              {-1, 1, 0}, {1, 0, 1},   {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                              {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
    return t[i][a];
}
template <>
__device__ constexpr int cq<15>(int i, int a) {
    constexpr int t[15][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                              {0, 0, 1},  {0, 0, -1}, {1, 1, 1},  {-1, 1, 1},  {1, -1, 1},
                              {-1, -1, 1}, {1, 1, -1}, {-1, 1, -1}, {1, -1, -1}, {-1, -1, -1}};
    return t[i][a];
}
template <int Q>
__device__ constexpr double wq(int i) {
    return Q == 19 ? (i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0))
                   : (i == 0 ? 2.0 / 9.0 : (i < 7 ? 1.0 / 9.0 : 1.0 / 72.0));
}

template <typename T>
struct Tile3 {};
#ifndef LKS_FWD3D_ZC
#define LKS_FWD3D_ZC 32
#endif
template <>
struct Tile3<float> {
    static constexpr int TX = 32, TY = 8, ZC = LKS_FWD3D_ZC;  // longest z chunk of a block
};
template <>
struct Tile3<double> {
    static constexpr int TX = 16, TY = 8, ZC = 32;
};

__device__ __forceinline__ int ring5(int z) { return ((z % 5) + 5) % 5; }
__device__ __forceinline__ int ring3(int z) { return ((z % 3) + 3) % 3; }

// derivative along one axis from five samples f(-2..2) around a node at coordinate c
template <typename T>
__device__ __forceinline__ T dcoord(T fm2, T fm1, T f0, T fp1, T fp2, int c, int n, int per) {
    if (!per && c == 0) return T(-1.5) * f0 + T(2) * fp1 - T(0.5) * fp2;
    if (!per && c == n - 1) return T(1.5) * f0 - T(2) * fm1 + T(0.5) * fm2;
    return T(0.5) * (fp1 - fm1);
}

// ================================== forward ==================================================
template <int Q>
__device__ constexpr int opp(int q) {  // index of -c_q
    for (int r = 0; r < Q; ++r)
        if (cq<Q>(r, 0) == -cq<Q>(q, 0) && cq<Q>(r, 1) == -cq<Q>(q, 1) && cq<Q>(r, 2) == -cq<Q>(q, 2)) return r;
    return q;
}

// face nodes written from interior node c3 (value v), with their objective contribution
template <typename T>
__device__ __noinline__ double fwd3d_push(const FwdArgs<T> &a, int x, int y, int z, T r, T u0, T u1,
                                          T u2, bool obj_on) {
    const Geom &g = a.g;
    double j = 0.0;
    const int c3[3] = {x, y, z};
    const T v[4] = {r, u0, u1, u2};
    push_boundary<T, 3>(g, a.bc, c3, v, [&](const int p[3], const T pv[4]) {
        const long long pi = p[0] + p[1] * g.sy + p[2] * g.sz;
        a.rout[pi] = pv[0];
        a.uout[0][pi] = pv[1];
        a.uout[1][pi] = pv[2];
        a.uout[2][pi] = pv[3];
        if (obj_on && !obj_uses_kappa(a.obj.kind) && (!a.obj.mask || a.obj.mask[pi])) {
            const T pu[3] = {pv[1], pv[2], pv[3]}, z3[3] = {0, 0, 0};
            j += obj_density<T>(a.obj, p[0], p[1], p[2], (double)pv[0], pu, T(0), z3);
        }
    });
    return j;
}

// one-sided second-order derivative at a face node: into the domain from f0 (lo) or (hi)
template <typename T>
__device__ __forceinline__ T d_lo(T f0, T f1, T f2) { return T(-1.5) * f0 + T(2) * f1 - T(0.5) * f2; }
template <typename T>
__device__ __forceinline__ T d_hi(T f0, T f1, T f2) { return T(1.5) * f0 - T(2) * f1 + T(0.5) * f2; }

// LDS of the z-marching forward: a ring of velocity planes (halo 2), then the E_i plane (halo 1)
// of every moving direction; the rest population E_0 is pulled only by its own node, which
// evaluates it itself.  Five velocity planes in general (one-sided z differences at z faces),
// three when the domain is periodic in z; with three, four blocks share a CU (FP32 D3Q19).
template <typename T, int Q>
struct Fwd3Lds {
    static constexpr int TX = Tile3<T>::TX, TY = Tile3<T>::TY;
    static constexpr int UX = TX + 4, UY = TY + 4, UP = UX * UY;
    static constexpr int EX = TX + 2, EY = TY + 2, EP = EX * EY;
    static constexpr size_t bytes(bool pz) { return (size_t)((pz ? 3 : 5) * 3 * UP + (Q - 1) * EP) * sizeof(T); }
};

template <bool PZ>
__device__ __forceinline__ int uring(int z) { return PZ ? ring3(z) : ring5(z); }

template <typename T, int Q, bool PZ>
__device__ __forceinline__ void fwd3d_body(const FwdArgs<T> &a, int bx, int by, int bz, long long blin, T *lds) {
    constexpr int TX = Tile3<T>::TX, TY = Tile3<T>::TY, NT = TX * TY;
    constexpr int UX = TX + 4, UY = TY + 4, UP = UX * UY;  // velocity plane, halo 2
    constexpr int EX = TX + 2, EY = TY + 2, EP = EX * EY;  // E_i plane, halo 1
    constexpr int NU = (UP + NT - 1) / NT, NE = (EP + NT - 1) / NT;
    constexpr int NR = PZ ? 3 : 5;  // velocity planes in the ring
    constexpr int LA = PZ ? 2 : 3;  // the plane committed after the E pass of plane zc is zc + LA
    T(*su)[3][UP] = reinterpret_cast<T(*)[3][UP]>(lds);
    T(*sE)[EP] = reinterpret_cast<T(*)[EP]>(lds + NR * 3 * UP);  // row q - 1 holds E_q
    __shared__ double sh[NT / 64];

    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY, zs = bz * g.zc;
    const int ze = min(zs + g.zc, nz);
    const T A = a.A;
    // block-uniform: E or output nodes of the block on or next to a non-periodic x / y face
    const bool xface = !g.per[0] && (x0 - 1 <= 1 || x0 + TX >= nx - 2);
    const bool yface = !g.per[1] && (y0 - 1 <= 1 || y0 + TY >= ny - 2);
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const bool kobj = obj_on && obj_uses_kappa(a.obj.kind);

    // per-thread offsets, computed once: velocity-plane slots (x, y wrapped; -1 off the domain)
    long long uoff[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        const int i = tid + k * NT;
        uoff[k] = -1;
        if (i >= UP) continue;
        int gx = x0 - 2 + i % UX, gy = y0 - 2 + i / UX;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1])) uoff[k] = gx + (long long)gy * g.sy;
    }
    // E slots: index of the node in a velocity plane, offset of its rho, face bits (1 x = 0,
    // 2 x = nx - 1, 4 y = 0, 8 y = ny - 1); -1 for slots off the domain (their E is never pulled)
    int ec0[NE], efl[NE];
    long long roff[NE];
#pragma unroll
    for (int k = 0; k < NE; ++k) {
        const int i = tid + k * NT;
        efl[k] = -1;
        ec0[k] = 0;
        roff[k] = 0;
        if (i >= EP) continue;
        const int lx = i % EX, ly = i / EX;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        if (!wrapc(gx, nx, g.per[0]) || !wrapc(gy, ny, g.per[1])) continue;
        ec0[k] = (ly + 1) * UX + (lx + 1);
        roff[k] = gx + (long long)gy * g.sy;
        int f = 0;
        if (!g.per[0]) f |= (gx == 0 ? 1 : 0) | (gx == nx - 1 ? 2 : 0);
        if (!g.per[1]) f |= (gy == 0 ? 4 : 0) | (gy == ny - 1 ? 8 : 0);
        efl[k] = f;
    }
    // this thread's output column
    const int ox = tid % TX, oy = tid / TX;
    const int gxo = x0 + ox, gyo = y0 + oy;
    const bool out_ok = gxo < nx && gyo < ny && !on_face(g, 0, gxo) && !on_face(g, 1, gyo);
    const long long ooff = gxo + (long long)gyo * g.sy;
    const bool xybox = a.m.hi[0] >= x0 && a.m.lo[0] < x0 + TX && a.m.hi[1] >= y0 && a.m.lo[1] < y0 + TY;
    const bool obox = out_ok && gxo >= a.m.lo[0] && gxo <= a.m.hi[0] && gyo >= a.m.lo[1] && gyo <= a.m.hi[1];
    const int per2 = g.per[2];

    // two register sets of velocity planes: the plane loaded in one iteration is committed to the
    // LDS ring in the next, so its loads have a whole iteration to arrive
    T ua[NU][3], ub[NU][3];
    T rreg[NE];
    // argument fields used in the loop, held locally: stores through the output pointers could
    // otherwise alias the argument block and force it to be re-read
    const LKS_GLOBAL T *__restrict__ uin0 = gld(a.uin[0]);
    const LKS_GLOBAL T *__restrict__ uin1 = gld(a.uin[1]);
    const LKS_GLOBAL T *__restrict__ uin2 = gld(a.uin[2]);
    const LKS_GLOBAL T *__restrict__ rin = gld(a.rin);
    LKS_GLOBAL T *__restrict__ rout = gst(a.rout);
    LKS_GLOBAL T *__restrict__ uout0 = gst(a.uout[0]);
    LKS_GLOBAL T *__restrict__ uout1 = gst(a.uout[1]);
    LKS_GLOBAL T *__restrict__ uout2 = gst(a.uout[2]);
    const LKS_GLOBAL T *__restrict__ kin = gld(a.kin);
    const LKS_GLOBAL T *__restrict__ usin0 = gld(a.usin[0]);
    const LKS_GLOBAL T *__restrict__ usin1 = gld(a.usin[1]);
    const LKS_GLOBAL T *__restrict__ usin2 = gld(a.usin[2]);
    const LKS_GLOBAL T *__restrict__ kst = gld(a.kstatic);
    const LKS_GLOBAL uint8_t *__restrict__ omask = gld(a.obj.mask);
    const StepMotion m = a.m;    // motion and box geometry of this step, held in registers
    const BoxGeom box = a.box;
    const T gf0 = a.gf[0], gf1 = a.gf[1], gf2 = a.gf[2];
    const long long sz = g.sz;
    // loads are unconditional (slots off the domain read element 0 and select zero), so the
    // wait counters can follow each load and a plane's loads overlap the previous plane's work
    auto fetch_u = [&](T(&ureg)[NU][3], int zp) {
        int zw = zp;
        const bool zin = wrapc(zw, nz, g.per[2]);
        const long long zo = zin ? (long long)zw * sz : 0;
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            const bool ok = zin && uoff[k] >= 0;
            const long long o = ok ? uoff[k] + zo : 0;
            const T v0 = uin0[o], v1 = uin1[o], v2 = uin2[o];
            ureg[k][0] = ok ? v0 : T(0);
            ureg[k][1] = ok ? v1 : T(0);
            ureg[k][2] = ok ? v2 : T(0);
        }
    };
    auto commit_u = [&](T(&ureg)[NU][3], int zp) {
        const int sl = uring<PZ>(zp);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            const int i = tid + k * NT;
            if (i < UP) {
                su[sl][0][i] = ureg[k][0];
                su[sl][1][i] = ureg[k][1];
                su[sl][2][i] = ureg[k][2];
            }
        }
    };
    auto fetch_r = [&](int zp) {
        int zw = zp;
        const bool zin = wrapc(zw, nz, g.per[2]);
        const long long zo = zin ? (long long)zw * sz : 0;
#pragma unroll
        for (int k = 0; k < NE; ++k) {
            const bool ok = zin && efl[k] >= 0;
            const T v = rin[ok ? roff[k] + zo : 0];
            rreg[k] = ok ? v : T(0);
        }
    };

    // the first E plane (zs - 1) reads velocity planes zs - 1 - NR / 2 .. zs - 1 + NR / 2
    for (int zp = zs - 1 - NR / 2; zp <= zs - 1 + NR / 2; ++zp) {
        fetch_u(ua, zp);
        commit_u(ua, zp);
    }
    fetch_r(zs - 1);
    fetch_u(ua, zs - 1 + LA);  // committed by the first iteration
    __syncthreads();
    const int own_u = (oy + 2) * UX + (ox + 2);  // this thread's output column in a velocity plane

    T acc[3][4];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = T(0);
    double jacc = 0.0;

    auto step = [&](int zc, T(&ucommit)[NU][3], T(&uload)[NU][3]) {
        const int zo = zc - 1;  // output plane finished in this iteration
        const bool zout = zo >= zs && zo < ze && !on_face(g, 2, zo);
        // footprint values and kappa_s of this thread's output node, requested early
        T kap = T(0), us0 = T(0), us1 = T(0), us2 = T(0), ks = T(0);
        if (xybox) {  // block-uniform
            const bool inb = zout && obox && zo >= m.lo[2] && zo <= m.hi[2];
            const long long bi = inb ? box_index(box, m, 3, gxo, gyo, zo) : 0;
            const T k0 = kin[bi], s0v = usin0[bi], s1v = usin1[bi], s2v = usin2[bi];
            kap = inb ? k0 : T(0);
            us0 = inb ? s0v : T(0);
            us1 = inb ? s1v : T(0);
            us2 = inb ? s2v : T(0);
        }
        if (kst) {  // block-uniform
            const bool ok = zout && out_ok;
            const T kv = kst[ok ? ooff + (long long)zo * sz : 0];
            ks = ok ? kv : T(0);
        }
        // rho - 1 of this thread's own node in plane zc, for its rest population
        int zwc = zc;
        const bool zinc = wrapc(zwc, nz, g.per[2]) && out_ok;
        const T rown_v = rin[zinc ? ooff + (long long)zwc * sz : 0];
        const T rown = zinc ? rown_v : T(0);
        T rcur[NE];
#pragma unroll
        for (int k = 0; k < NE; ++k) rcur[k] = rreg[k];
        fetch_u(uload, zc + 1 + LA);  // committed by the next iteration
        fetch_r(zc + 1);
        int zw = zc;
        const bool zin = wrapc(zw, nz, g.per[2]);
        // E of every slot of plane zc.  FACE: some slot of the block may sit on a non-periodic
        // face (one-sided derivatives); blocks away from every face take the straight-line code,
        // whose LDS reads are all issued before the arithmetic
        auto e_pass = [&](auto face_tag) {
            constexpr bool FACE = decltype(face_tag)::value;
            // (planes zc +- 2 only for the one-sided rows at z faces, never in a z-periodic ring)
            const int s0 = uring<PZ>(zc), sm1 = uring<PZ>(zc - 1), sp1 = uring<PZ>(zc + 1),
                      sm2 = uring<PZ>(zc - 2), sp2 = uring<PZ>(zc + 2);
            const bool zlo = !g.per[2] && zw == 0, zhi = !g.per[2] && zw == nz - 1;
#pragma unroll
            for (int k = 0; k < NE; ++k) {
                if (efl[k] < 0) continue;
                const int c0 = ec0[k];
                T u[3], du[3][3];  // du[c][b] = d u_c / d x_b
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T *p = su[s0][c];
                    u[c] = p[c0];
                    du[c][0] = T(0.5) * (p[c0 + 1] - p[c0 - 1]);
                    du[c][1] = T(0.5) * (p[c0 + UX] - p[c0 - UX]);
                    du[c][2] = T(0.5) * (su[sp1][c][c0] - su[sm1][c][c0]);
                    if constexpr (FACE) {
                        if (xface && (efl[k] & 3))
                            du[c][0] = (efl[k] & 1) ? d_lo(u[c], p[c0 + 1], p[c0 + 2]) : d_hi(u[c], p[c0 - 1], p[c0 - 2]);
                        if (yface && (efl[k] & 12))
                            du[c][1] = (efl[k] & 4) ? d_lo(u[c], p[c0 + UX], p[c0 + 2 * UX])
                                                    : d_hi(u[c], p[c0 - UX], p[c0 - 2 * UX]);
                        if (zlo) du[c][2] = d_lo(u[c], su[sp1][c][c0], su[sp2][c][c0]);
                        if (zhi) du[c][2] = d_hi(u[c], su[sm1][c][c0], su[sm2][c][c0]);
                    }
                }
                const T a0 = rcur[k] - T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                T tt[3][3];
#pragma unroll
                for (int pp = 0; pp < 3; ++pp)
#pragma unroll
                    for (int qq = pp; qq < 3; ++qq)
                        tt[pp][qq] = T(4.5) * u[pp] * u[qq] + A * (du[pp][qq] + du[qq][pp]);
                const int i = tid + k * NT;
                // +c and -c share the even part a0 + c.T.c; the odd part 3 c.u changes sign
#pragma unroll
                for (int q = 1; q < Q; ++q) {
                    if (opp<Q>(q) < q) continue;
                    const int cx = cq<Q>(q, 0), cy = cq<Q>(q, 1), cz = cq<Q>(q, 2);
                    // c.T.c and c.u over the non-zero components of c only (|c_b| <= 1): a product
                    // with a zero coefficient is not folded away in IEEE arithmetic
                    T ev = a0;
                    if (cx) ev += tt[0][0];
                    if (cy) ev += tt[1][1];
                    if (cz) ev += tt[2][2];
                    if (cx && cy) ev += T(2 * cx * cy) * tt[0][1];
                    if (cx && cz) ev += T(2 * cx * cz) * tt[0][2];
                    if (cy && cz) ev += T(2 * cy * cz) * tt[1][2];
                    // (built from its first non-zero term: 0 + x is not folded to x either)
                    T cu = cx ? T(cx) * u[0] : T(0);
                    if (cy) cu = cx ? cu + T(cy) * u[1] : T(cy) * u[1];
                    if (cz) cu = (cx || cy) ? cu + T(cz) * u[2] : T(cz) * u[2];
                    const T od = T(3) * cu;
                    sE[q - 1][i] = T(wq<Q>(q)) * (ev + od);
                    sE[opp<Q>(q) - 1][i] = T(wq<Q>(q)) * (ev - od);
                }
            }
        };
        if (zin) {
            const bool zface = !g.per[2] && (zw == 0 || zw == nz - 1);
            if (xface || yface || zface) e_pass(std::true_type{});
            else e_pass(std::false_type{});
        }
        // the rest population of the own node, from its own rho and u (the commit below
        // replaces plane zc - NR / 2, not plane zc)
        T e0 = T(0);
        if (zin) {
            const T u0 = su[uring<PZ>(zc)][0][own_u], u1 = su[uring<PZ>(zc)][1][own_u];
            const T u2 = su[uring<PZ>(zc)][2][own_u];
            e0 = T(wq<Q>(0)) * (rown - T(1.5) * (u0 * u0 + u1 * u1 + u2 * u2));
        }
        __syncthreads();
        commit_u(ucommit, zc + LA);
        // pull: output (x, y, zo) takes E_i from (x - cx, y - cy) in plane zo - cz
        if (zin) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int cx = cq<Q>(q, 0), cy = cq<Q>(q, 1), cz = cq<Q>(q, 2);
                const T e = q == 0 ? e0 : sE[q - 1][(oy + 1 - cy) * EX + (ox + 1 - cx)];
                const int t = cz + 1;  // cz = -1 -> plane zc - 1, 0 -> zc, +1 -> zc + 1
                acc[t][0] += e;
                if (cx) acc[t][1] += T(cx) * e;
                if (cy) acc[t][2] += T(cy) * e;
                if (cz) acc[t][3] += T(cz) * e;
            }
        }
        if (zout && out_ok) {
            const T rs = acc[0][0];
            T nu0 = acc[0][1] + gf0, nu1 = acc[0][2] + gf1, nu2 = acc[0][3] + gf2;
            if (xybox || kst) {
                const T inv = T(1) / (T(1) + kap + ks);
                nu0 = (nu0 + kap * us0) * inv;
                nu1 = (nu1 + kap * us1) * inv;
                nu2 = (nu2 + kap * us2) * inv;
            }
            const long long idx = ooff + (long long)zo * sz;
            rout[idx] = rs;
            uout0[idx] = nu0;
            uout1[idx] = nu1;
            uout2[idx] = nu2;
            if (obj_on && (!kobj || kap != T(0)) && (!omask || omask[idx])) {
                const T nu[3] = {nu0, nu1, nu2}, us[3] = {us0, us1, us2};
                jacc += obj_density<T>(a.obj, gxo, gyo, zo, (double)rs, nu, kap, us);
            }
            const bool zadj = !per2 && (zo == 1 || zo == nz - 2);
            if (xface && !yface && !zadj) {  // block- and plane-uniform: only an x face is in reach
                if (gxo == 1 || gxo == nx - 2) {  // the face node next to this one, by that face's rule
                    const int f = gxo == 1 ? 0 : 1, kind = a.bc.kind[f], pc = gxo == 1 ? 0 : nx - 1;
                    const T pr = bc_copies(kind, 0, 0) ? rs : a.bc.rho[f];
                    const T p0 = bc_copies(kind, 1, 0) ? nu0 : a.bc.u[f][0];
                    const T p1 = bc_copies(kind, 2, 0) ? nu1 : a.bc.u[f][1];
                    const T p2 = bc_copies(kind, 3, 0) ? nu2 : a.bc.u[f][2];
                    const long long pi = pc + (long long)gyo * g.sy + (long long)zo * sz;
                    rout[pi] = pr;
                    uout0[pi] = p0;
                    uout1[pi] = p1;
                    uout2[pi] = p2;
                    if (obj_on && !kobj && (!omask || omask[pi])) {
                        const T pu[3] = {p0, p1, p2}, z3[3] = {T(0), T(0), T(0)};
                        jacc += obj_density<T>(a.obj, pc, gyo, zo, (double)pr, pu, T(0), z3);
                    }
                }
            } else if ((xface && (gxo == 1 || gxo == nx - 2)) || (yface && (gyo == 1 || gyo == ny - 2)) || zadj) {
                jacc += fwd3d_push<T>(a, gxo, gyo, zo, rs, nu0, nu1, nu2, obj_on);
            }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[0][c] = acc[1][c];
            acc[1][c] = acc[2][c];
            acc[2][c] = T(0);
        }
        __syncthreads();
    };
    for (int zc = zs - 1; zc <= ze; zc += 2) {
        step(zc, ua, ub);
        if (zc + 1 <= ze) step(zc + 1, ub, ua);
    }
    if (obj_on) store_partial<NT>(a.obj, jacc, blin, sh);
}

__device__ __forceinline__ int job_of3(const long long *tile0, int njobs, long long b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

#ifndef LKS_XCD3D
#define LKS_XCD3D 1
#endif
// column (bx, by) and z chunk bz of the t-th dispatched block: each XCD takes a contiguous run of
// tiles (x fastest), so blocks that share x-y halo planes read them through one L2
template <typename T>
__device__ __forceinline__ void tile_coords3(const Geom &g, int zc, long long t, int &bx, int &by, int &bz) {
    const int nbx = (g.n[0] + Tile3<T>::TX - 1) / Tile3<T>::TX;
    const int nby = (g.n[1] + Tile3<T>::TY - 1) / Tile3<T>::TY;
#if LKS_XCD3D
    const unsigned tu = (unsigned)xcd_tile(t, (long long)nbx * nby * ((g.n[2] + zc - 1) / zc));
#else
    const unsigned tu = (unsigned)t;
#endif
    bx = (int)(tu % (unsigned)nbx);
    by = (int)((tu / (unsigned)nbx) % (unsigned)nby);
    bz = (int)(tu / ((unsigned)nbx * (unsigned)nby));
}

template <typename T>
__device__ __forceinline__ long long stencil_tiles3(const Geom &g) {
    return (long long)((g.n[0] + Tile3<T>::TX - 1) / Tile3<T>::TX) *
           ((g.n[1] + Tile3<T>::TY - 1) / Tile3<T>::TY) * ((g.n[2] + g.zc - 1) / g.zc);
}

// PZ: every job of the launch is periodic in z (the three-plane velocity ring; dynamic LDS sized
// to it).  One kernel per layout, so each gets its own register allocation.
template <typename T, int Q, bool PZ>
__global__ __launch_bounds__(Tile3<T>::TX * Tile3<T>::TY) void k_fwd3d_batch(const FwdArgs<T> *__restrict__ args,
                                                                            const long long *__restrict__ tile0,
                                                                            int njobs) {
    extern __shared__ __align__(16) unsigned char fwd3_lds[];
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of3(tile0, njobs, b));
    const FwdArgs<T> &a = args[j];
    const long long t = njobs == 1 ? b : b - tile0[j];  // one job: tile0 = {0}
    const long long ns = (a.mode & FWD_STENCIL) ? stencil_tiles3<T>(a.g) : 0;
    if (t >= ns) {  // extra blocks: transfer of the next step onto its footprint box
        transfer_box<T, 3, Tile3<T>::TX * Tile3<T>::TY>(a.des, a.mnext, a.box, a.knext, a.usnext, t - ns);
        return;
    }
    int bx, by, bz;
    tile_coords3<T>(a.g, a.g.zc, t, bx, by, bz);
    fwd3d_body<T, Q, PZ>(a, bx, by, bz, t, reinterpret_cast<T *>(fwd3_lds));
}

// ================================== adjoint, pointwise part ===================================
// lambda = Lambda + dj/dX at one node (kappa = 0 and u_S = 0 outside the footprint box)
template <typename T>
__device__ __forceinline__ void lambda_at(const AdjArgs<T> &a, int x, int y, int z, long long idx,
                                          T lam[4]) {
    lam[0] = a.Pin[idx];
    lam[1] = a.Vin[0][idx];
    lam[2] = a.Vin[1][idx];
    lam[3] = a.Vin[2][idx];
    if (!(a.obj.active && a.obj.kind != OBJ_NONE)) return;
    if (a.obj.mask && !a.obj.mask[idx]) return;
    double kap = 0.0, us[3] = {0, 0, 0};
    if (obj_uses_kappa(a.obj.kind) && in_box(a.m, 3, x, y, z)) {
        const long long bi = box_index(a.box, a.m, 3, x, y, z);
        kap = a.kbox[bi];
        us[0] = a.usbox[0][bi];
        us[1] = a.usbox[1][bi];
        us[2] = a.usbox[2][bi];
    }
    double dP, dV[3];
    obj_dstate(a.obj, x, y, z, kap, us, dP, dV);
    const double sc = a.obj.scale;
    lam[0] += (T)(sc * dP);
    lam[1] += (T)(sc * dV[0]);
    lam[2] += (T)(sc * dV[1]);
    lam[3] += (T)(sc * dV[2]);
}

// Row fast path of the pointwise part: the wave's 64 nodes are consecutive in x within one (y, z)
// row that is neither on nor next to a non-periodic y or z face.  The only boundary rule that can
// reach them is an x face inside the wave: face nodes hold P* = V* = 0 and the node next to a face
// takes that face's seed through one lane shift, per component as the face's rule copies it
// (the wave holds the face whenever it holds the node next to it; the caller checks).
template <typename T>
__device__ __forceinline__ void adj3d_prep_row(const AdjArgs<T> &a, int x0, int y, int z) {
    const Geom &g = a.g;
    const int lane = threadIdx.x & 63;
    const int x = x0 + lane, nx = g.n[0];
    const long long idx = x + y * g.sy + z * g.sz;
    T lam[4] = {a.Pin[idx], a.Vin[0][idx], a.Vin[1][idx], a.Vin[2][idx]};
    // footprint values of the row: one clamped load per lane when the row meets the box
    const bool rbox = y >= a.m.lo[1] && y <= a.m.hi[1] && z >= a.m.lo[2] && z <= a.m.hi[2] &&
                      a.m.hi[0] >= x0 && a.m.lo[0] <= x0 + 63;
    const bool inb = rbox && x >= a.m.lo[0] && x <= a.m.hi[0];
    T kap = T(0), us[3] = {T(0), T(0), T(0)}, uc[3] = {T(0), T(0), T(0)};
    long long bi = 0;
    if (rbox) {  // wave-uniform
        const int xc = min(max(x, a.m.lo[0]), a.m.hi[0]);
        bi = box_index(a.box, a.m, 3, xc, y, z);
        const long long ic = xc + y * g.sy + z * g.sz;  // a box node: inside the grid
        const T k0 = a.kbox[bi], s0 = a.usbox[0][bi], s1 = a.usbox[1][bi], s2 = a.usbox[2][bi];
        const T c0 = a.ucur[0][ic], c1 = a.ucur[1][ic], c2 = a.ucur[2][ic];
        kap = inb ? k0 : T(0);
        us[0] = inb ? s0 : T(0);
        us[1] = inb ? s1 : T(0);
        us[2] = inb ? s2 : T(0);
        uc[0] = c0;
        uc[1] = c1;
        uc[2] = c2;
    }
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const bool kobj = obj_on && obj_uses_kappa(a.obj.kind);
    if (obj_on && (rbox || !kobj)) {  // kappa objectives vanish off the footprint
        const bool mk = !a.obj.mask || a.obj.mask[idx];
        if (mk && !(kobj && kap == T(0))) {
            const double usd[3] = {(double)us[0], (double)us[1], (double)us[2]};
            double dP, dV[3];
            obj_dstate(a.obj, x, y, z, (double)kap, usd, dP, dV);
            const double sc = a.obj.scale;
            lam[0] += (T)(sc * dP);
            lam[1] += (T)(sc * dV[0]);
            lam[2] += (T)(sc * dV[1]);
            lam[3] += (T)(sc * dV[2]);
        }
    }
    if (!g.per[0]) {  // the x faces
        const int kl = a.bc.kind[0], kr = a.bc.kind[1];
        const bool nl = x == 1, nr = x == nx - 2;
        T sh[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T fl = from_left(lam[c]), fr = from_right(lam[c]);
            sh[c] = (nl && bc_copies(kl, c, 0) ? fl : T(0)) + (nr && bc_copies(kr, c, 0) ? fr : T(0));
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) lam[c] += sh[c];
        if (x == 0 || x == nx - 1) lam[0] = lam[1] = lam[2] = lam[3] = T(0);
    }
    const T ks = a.kstatic ? a.kstatic[idx] : T(0);
    const T inv = T(1) / (T(1) + kap + ks);
    const T V[3] = {lam[1] * inv, lam[2] * inv, lam[3] * inv};
    a.Ps[idx] = lam[0];
    a.Vs[0][idx] = V[0];
    a.Vs[1][idx] = V[1];
    a.Vs[2][idx] = V[2];
    if (inb) {
        double uu[3], uss[3];
        double kb = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uu[k] = (double)uc[k];
            uss[k] = (double)us[k];
            kb -= (double)V[k] * (uu[k] - uss[k]);
        }
        if (kobj && (!a.obj.mask || a.obj.mask[idx]))
            kb += a.obj.scale * obj_dkappa(a.obj, x, y, z, uu, uss);
        a.kbar[bi] = (T)kb;
    }
}

// One node of the pointwise part, any boundary configuration (t: the node's linear index)
template <typename T>
__device__ __forceinline__ void adj3d_prep_node(const AdjArgs<T> &a, long long t) {
    const Geom &g = a.g;
    const unsigned tu = (unsigned)t, n0 = (unsigned)g.n[0], n1 = (unsigned)g.n[1];  // < 2^31 cells
    const int x = (int)(tu % n0), y = (int)((tu / n0) % n1), z = (int)(tu / (n0 * n1));
    const long long idx = x + y * g.sy + z * g.sz;
    if (on_face(g, 0, x) || on_face(g, 1, y) || on_face(g, 2, z)) {
        a.Ps[idx] = T(0);
        a.Vs[0][idx] = a.Vs[1][idx] = a.Vs[2][idx] = T(0);
        return;
    }
    T lam[4];
    lambda_at(a, x, y, z, idx, lam);
    const int c[3] = {x, y, z};
    gather_boundary_T<3>(g, a.bc.kind, c, lam, [&](const int p[3], int comp) -> T {
        T lp[4];
        lambda_at(a, p[0], p[1], p[2], p[0] + p[1] * g.sy + p[2] * g.sz, lp);
        return comp == 0 ? lp[0] : comp == 1 ? lp[1] : comp == 2 ? lp[2] : lp[3];
    });
    T kap = 0, us[3] = {0, 0, 0};
    const bool inb = in_box(a.m, 3, x, y, z);
    long long bi = 0;
    if (inb) {
        bi = box_index(a.box, a.m, 3, x, y, z);
        kap = a.kbox[bi];
        us[0] = a.usbox[0][bi];
        us[1] = a.usbox[1][bi];
        us[2] = a.usbox[2][bi];
    }
    const T ks = a.kstatic ? a.kstatic[idx] : T(0);
    const T inv = T(1) / (T(1) + kap + ks);
    const T V[3] = {lam[1] * inv, lam[2] * inv, lam[3] * inv};
    a.Ps[idx] = lam[0];
    a.Vs[0][idx] = V[0];
    a.Vs[1][idx] = V[1];
    a.Vs[2][idx] = V[2];
    if (inb) {
        double uu[3], uss[3];
        double kb = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uu[k] = (double)a.ucur[k][idx];
            uss[k] = (double)us[k];
            kb -= (double)V[k] * (uu[k] - uss[k]);
        }
        if (a.obj.active && obj_uses_kappa(a.obj.kind) && (!a.obj.mask || a.obj.mask[idx]))
            kb += a.obj.scale * obj_dkappa(a.obj, x, y, z, uu, uss);
        a.kbar[bi] = (T)kb;
    }
}

// A wave takes prep_rows3(ncell) consecutive 64-node segments of the linear node order, so its
// uniform work (argument loads, the segment's coordinates, the fast-path test) is paid once per
// segment with coordinates advanced by additions instead of divisions.
template <typename T>
__device__ __forceinline__ void adj3d_prep_body(const AdjArgs<T> &a, long long blk) {
    const Geom &g = a.g;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    const int rows = prep_rows3(ncell);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    long long tw = (blk * (kBlock / 64) + wave) * 64LL * rows;
    if (tw >= ncell) return;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const unsigned n0 = (unsigned)nx, n1 = (unsigned)ny;
    int x0, y, z;
    {
        const unsigned twu = (unsigned)tw;  // < 2^31 cells
        x0 = (int)(twu % n0);
        y = (int)((twu / n0) % n1);
        z = (int)(twu / (n0 * n1));
    }
    const int lane = threadIdx.x & 63;
    for (int r = 0; r < rows && tw < ncell; ++r, tw += 64) {
        // wave-uniform row test for the fast path
        const bool row = tw + 63 < ncell && x0 + 63 < nx;
        const bool yok = g.per[1] || (y >= 2 && y <= ny - 3);
        const bool zok = g.per[2] || (z >= 2 && z <= nz - 3);
        const bool xok = g.per[0] || (x0 != 1 && x0 + 63 != nx - 2);  // a face next to the wave's ends
        if (row && yok && zok && xok) adj3d_prep_row<T>(a, x0, y, z);
        else if (tw + lane < ncell) adj3d_prep_node<T>(a, tw + lane);
        x0 += 64;
        while (x0 >= nx) {
            x0 -= nx;
            if (++y == ny) {
                y = 0;
                ++z;
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj3d_prep_batch(const AdjArgs<T> *__restrict__ args,
                                                             const long long *__restrict__ blk0, int njobs) {
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of3(blk0, njobs, b));
    adj3d_prep_body<T>(args[j], njobs == 1 ? b : b - blk0[j]);
}

// ================================== adjoint, z-marching part ==================================
template <typename T>
__device__ __forceinline__ T deriv_T3(const T f[5], int c, int n, int per) {
    if (per) return T(0.5) * (f[1] - f[3]);
    T acc = 0;
#pragma unroll
    for (int o = -2; o <= 2; ++o) {
        const int r = c + o;
        if (r < 0 || r >= n) continue;
        T coef = 0;
        if (r == 0) coef = (c == 0) ? T(-1.5) : (c == 1) ? T(2) : (c == 2) ? T(-0.5) : T(0);
        else if (r == n - 1) coef = (c == n - 1) ? T(1.5) : (c == n - 2) ? T(-2) : (c == n - 3) ? T(0.5) : T(0);
        else coef = (c == r + 1) ? T(0.5) : (c == r - 1) ? T(-0.5) : T(0);
        acc += coef * f[o + 2];
    }
    return acc;
}

// LDS of the z-marching adjoint: three (P*, V*) planes with halo 3, then s~ planes (halo 2).  A
// domain that is not periodic in z keeps a ring of five planes of all six s~ components (the
// transposed one-sided rows at the z faces read two planes each way; outputs lag the moments by
// two planes).  A z-periodic domain needs only the central difference along z, which reads the
// output column's own s~ xz, yz, zz one plane each way: those three stay in the column thread's
// registers (planes zm - 2 .. zm), and LDS holds one plane of s~ xx, yy, xy, xz, yz (the
// components some x or y derivative reads from a neighbour), written after the output pass has
// read the previous one.  That is 34 KB in FP32, so four blocks share a CU (51 KB and three with
// a three-plane LDS ring).
template <typename T>
struct Adj3Lds {
    static constexpr int TX = Tile3<T>::TX, TY = Tile3<T>::TY;
    static constexpr int PX = TX + 6, PY = TY + 6, PP = PX * PY;  // (P*, V*) plane, halo 3
    static constexpr int MX = TX + 4, MY = TY + 4, MP = MX * MY;  // moment plane, halo 2
    static constexpr int SPV = 3 * 4 * PP;
    static constexpr size_t bytes(bool pz) { return (size_t)(SPV + (pz ? 5 : 30) * MP) * sizeof(T); }
};

// s~ component c (xx, yy, zz, xy, xz, yz) of moment plane z in the ring
template <typename T, bool PZ>
__device__ __forceinline__ T *s_plane(T *ss, int c, int z) {
    constexpr int MP = Adj3Lds<T>::MP;
    if (!PZ) return ss + (ring5(z) * 6 + c) * MP;
    // z-periodic: one plane of xx, yy, xy, xz, yz (zz is never read from LDS)
    (void)z;
    return ss + (c < 2 ? c : c - 1) * MP;
}

template <typename T, int Q, bool PZ>
__device__ __forceinline__ void adj3d_main_body(const AdjArgs<T> &a, int bx, int by, int bz, T *lds) {
    using L = Adj3Lds<T>;
    constexpr int TX = L::TX, TY = L::TY, NT = TX * TY;
    constexpr int PX = L::PX, PP = L::PP, MX = L::MX, MP = L::MP;
    constexpr int NP = (PP + NT - 1) / NT;
    constexpr int NH = MP - NT;  // halo moment nodes
    constexpr int LAG = PZ ? 1 : 2;  // output plane = moment plane - LAG
    static_assert(NH <= NT, "one halo pass");
    T(*spv)[4][PP] = reinterpret_cast<T(*)[4][PP]>(lds);
    T *ss = lds + L::SPV;

    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY, zs = bz * g.zca;
    const int ze = min(zs + g.zca, nz);
    const int ox = tid % TX, oy = tid / TX;

    // (P*, V*) plane slots of this thread (x, y wrapped; -1 off the domain), computed once
    long long poff[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) {
        const int i = tid + k * NT;
        poff[k] = -1;
        if (i >= PP) continue;
        int gx = x0 - 3 + i % PX, gy = y0 - 3 + i / PX;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1])) poff[k] = gx + (long long)gy * g.sy;
    }
    const LKS_GLOBAL T *__restrict__ ps = gld(a.Ps);
    const LKS_GLOBAL T *__restrict__ vs0 = gld(a.Vs[0]);
    const LKS_GLOBAL T *__restrict__ vs1 = gld(a.Vs[1]);
    const LKS_GLOBAL T *__restrict__ vs2 = gld(a.Vs[2]);
    const LKS_GLOBAL T *__restrict__ up0 = gld(a.uprev[0]);
    const LKS_GLOBAL T *__restrict__ up1 = gld(a.uprev[1]);
    const LKS_GLOBAL T *__restrict__ up2 = gld(a.uprev[2]);
    LKS_GLOBAL T *__restrict__ pout = gst(a.Pout);
    LKS_GLOBAL T *__restrict__ vout0 = gst(a.Vout[0]);
    LKS_GLOBAL T *__restrict__ vout1 = gst(a.Vout[1]);
    LKS_GLOBAL T *__restrict__ vout2 = gst(a.Vout[2]);
    const long long sz = g.sz;
    // loads are unconditional (slots off the domain read element 0 and select zero), so a plane's
    // loads stay in flight across the moment pass instead of draining where a branch rejoins
    T preg[NP][4];
    auto fetch_pv = [&](int zp) {
        int zw = zp;
        const bool zin = wrapc(zw, nz, g.per[2]);
        const long long zo = zin ? (long long)zw * sz : 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const bool ok = zin && poff[k] >= 0;
            const long long o = ok ? poff[k] + zo : 0;
            const T v0 = ps[o], v1 = vs0[o], v2 = vs1[o], v3 = vs2[o];
            preg[k][0] = ok ? v0 : T(0);
            preg[k][1] = ok ? v1 : T(0);
            preg[k][2] = ok ? v2 : T(0);
            preg[k][3] = ok ? v3 : T(0);
        }
    };
    auto commit_pv = [&](int zp) {
        const int sl = ring3(zp);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int i = tid + k * NT;
            if (i < PP)
#pragma unroll
                for (int c = 0; c < 4; ++c) spv[sl][c][i] = preg[k][c];
        }
    };
    // moments of the pull transpose at moment-plane node (lx, ly) of plane zm: with
    // e_q = P*(x + c_q) + c_q.V*(x + c_q), rho~ = sum w_q e_q, u~ = sum w_q c_q e_q and
    // s~_ab = sum w_q c_qa c_qb e_q.  The directions are summed by kind: a +-pair along an axis gives
    // its sum and difference, the four edges of a coordinate plane (D3Q19) and the eight corners
    // (D3Q15) their sums with every sign pattern (butterflies), so each e_q is formed once and
    // each moment is a short combination of these sums
    auto moments = [&](int zm, int lx, int ly, T m[10]) {
        const int s0 = ring3(zm), sm = ring3(zm - 1), sp = ring3(zm + 1);
        const int b0 = (ly + 1) * PX + (lx + 1);
        auto P = [&](int sl, int dx, int dy) -> T { return spv[sl][0][b0 + dy * PX + dx]; };
        auto V = [&](int sl, int c, int dx, int dy) -> T { return spv[sl][1 + c][b0 + dy * PX + dx]; };
        const T w0 = T(wq<Q>(0)), w1 = T(wq<Q>(1));
        const T fxp = P(s0, 1, 0) + V(s0, 0, 1, 0), fxm = P(s0, -1, 0) - V(s0, 0, -1, 0);
        const T fyp = P(s0, 0, 1) + V(s0, 1, 0, 1), fym = P(s0, 0, -1) - V(s0, 1, 0, -1);
        const T fzp = P(sp, 0, 0) + V(sp, 2, 0, 0), fzm = P(sm, 0, 0) - V(sm, 2, 0, 0);
        const T sfx = fxp + fxm, dfx = fxp - fxm, sfy = fyp + fym, dfy = fyp - fym;
        const T sfz = fzp + fzm, dfz = fzp - fzm;
        const T p0 = P(s0, 0, 0);
        // the four sums of e(+ +), e(+ -), e(- +), e(- -) with signs 1, s_a, s_b, s_a s_b
        auto quad = [](T epp, T epm, T emp, T emm, T &S, T &Sa, T &Sb, T &Sab) {
            const T a = epp + epm, bb = emp + emm, c = epp - epm, d = emp - emm;
            S = a + bb;
            Sa = a - bb;
            Sb = c + d;
            Sab = c - d;
        };
        if constexpr (Q == 19) {
            const T w2 = T(wq<Q>(7));
            T xy, xy_x, xy_y, xy_xy, xz, xz_x, xz_z, xz_xz, yz, yz_y, yz_z, yz_yz;
            {   // edges (+-1, +-1, 0): plane zm
                const T epp = P(s0, 1, 1) + V(s0, 0, 1, 1) + V(s0, 1, 1, 1);
                const T epm = P(s0, 1, -1) + V(s0, 0, 1, -1) - V(s0, 1, 1, -1);
                const T emp = P(s0, -1, 1) - V(s0, 0, -1, 1) + V(s0, 1, -1, 1);
                const T emm = P(s0, -1, -1) - V(s0, 0, -1, -1) - V(s0, 1, -1, -1);
                quad(epp, epm, emp, emm, xy, xy_x, xy_y, xy_xy);
            }
            {   // edges (+-1, 0, +-1): planes zm +- 1
                const T epp = P(sp, 1, 0) + V(sp, 0, 1, 0) + V(sp, 2, 1, 0);
                const T epm = P(sm, 1, 0) + V(sm, 0, 1, 0) - V(sm, 2, 1, 0);
                const T emp = P(sp, -1, 0) - V(sp, 0, -1, 0) + V(sp, 2, -1, 0);
                const T emm = P(sm, -1, 0) - V(sm, 0, -1, 0) - V(sm, 2, -1, 0);
                quad(epp, epm, emp, emm, xz, xz_x, xz_z, xz_xz);
            }
            {   // edges (0, +-1, +-1)
                const T epp = P(sp, 0, 1) + V(sp, 1, 0, 1) + V(sp, 2, 0, 1);
                const T epm = P(sm, 0, 1) + V(sm, 1, 0, 1) - V(sm, 2, 0, 1);
                const T emp = P(sp, 0, -1) - V(sp, 1, 0, -1) + V(sp, 2, 0, -1);
                const T emm = P(sm, 0, -1) - V(sm, 1, 0, -1) - V(sm, 2, 0, -1);
                quad(epp, epm, emp, emm, yz, yz_y, yz_z, yz_yz);
            }
            m[0] = w0 * p0 + w1 * (sfx + sfy + sfz) + w2 * (xy + xz + yz);
            m[1] = w1 * dfx + w2 * (xy_x + xz_x);
            m[2] = w1 * dfy + w2 * (xy_y + yz_y);
            m[3] = w1 * dfz + w2 * (xz_z + yz_z);
            m[4] = w1 * sfx + w2 * (xy + xz);
            m[5] = w1 * sfy + w2 * (xy + yz);
            m[6] = w1 * sfz + w2 * (xz + yz);
            m[7] = w2 * xy_xy;
            m[8] = w2 * xz_xz;
            m[9] = w2 * yz_yz;
        } else {  // D3Q15: the eight corners (+-1, +-1, +-1)
            const T w3 = T(wq<Q>(7));
            T S[2], Sx[2], Sy[2], Sxy[2];  // per z sign (0: +1, 1: -1)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int sl = h == 0 ? sp : sm;
                const T sz = h == 0 ? T(1) : T(-1);
                const T epp = P(sl, 1, 1) + V(sl, 0, 1, 1) + V(sl, 1, 1, 1) + sz * V(sl, 2, 1, 1);
                const T epm = P(sl, 1, -1) + V(sl, 0, 1, -1) - V(sl, 1, 1, -1) + sz * V(sl, 2, 1, -1);
                const T emp = P(sl, -1, 1) - V(sl, 0, -1, 1) + V(sl, 1, -1, 1) + sz * V(sl, 2, -1, 1);
                const T emm = P(sl, -1, -1) - V(sl, 0, -1, -1) - V(sl, 1, -1, -1) + sz * V(sl, 2, -1, -1);
                quad(epp, epm, emp, emm, S[h], Sx[h], Sy[h], Sxy[h]);
            }
            const T c = S[0] + S[1], cx = Sx[0] + Sx[1], cy = Sy[0] + Sy[1], cz = S[0] - S[1];
            const T cxz = Sx[0] - Sx[1], cyz = Sy[0] - Sy[1], cxy = Sxy[0] + Sxy[1];
            m[0] = w0 * p0 + w1 * (sfx + sfy + sfz) + w3 * c;
            m[1] = w1 * dfx + w3 * cx;
            m[2] = w1 * dfy + w3 * cy;
            m[3] = w1 * dfz + w3 * cz;
            m[4] = w1 * sfx + w3 * c;
            m[5] = w1 * sfy + w3 * c;
            m[6] = w1 * sfz + w3 * c;
            m[7] = w3 * cxy;
            m[8] = w3 * cxz;
            m[9] = w3 * cyz;
        }
    };

    const int zfirst = zs - LAG;  // first moment plane
    for (int zp = zfirst - 1; zp <= zfirst + 1; ++zp) {
        fetch_pv(zp);
        commit_pv(zp);
    }
    __syncthreads();
    T ru[3][4];  // rho~, u~ of the own column for planes zm-2, zm-1, zm
#pragma unroll
    for (int t = 0; t < 3; ++t) ru[t][0] = ru[t][1] = ru[t][2] = ru[t][3] = T(0);
    // z-periodic layout: s~ xz, yz, zz of the own column for planes zm-2, zm-1, zm, and this
    // plane's LDS components (xx, yy, xy, xz, yz) of the own column and of the halo node, stored
    // after the output pass
    T zr[3][3], own5[5], halo5[5];
    int hidx = 0;
#pragma unroll
    for (int t = 0; t < 3; ++t) zr[t][0] = zr[t][1] = zr[t][2] = T(0);
#pragma unroll
    for (int c = 0; c < 5; ++c) own5[c] = halo5[c] = T(0);
    const T A2 = T(2) * a.A;

    // transposed x- and y-derivatives of s~ at this thread's output column: central where every
    // column (row) of the block is at least three nodes from a face (or the axis is periodic),
    // else through coefficients that depend on the column (row) only, formed once here
    const int gxo = x0 + ox, gyo = y0 + oy;
    const bool xcen = g.per[0] || (x0 >= 3 && x0 + TX <= nx - 3);  // block-uniform
    const bool ycen = g.per[1] || (y0 >= 3 && y0 + TY <= ny - 3);
    T dcx[5], dcy[5];
#pragma unroll
    for (int o = 0; o < 5; ++o) {
        T f[5] = {T(0), T(0), T(0), T(0), T(0)};
        f[o] = T(1);
        dcx[o] = deriv_T3(f, gxo, nx, g.per[0]);
        dcy[o] = deriv_T3(f, gyo, ny, g.per[1]);
    }

    const bool col_ok = gxo < nx && gyo < ny;
    const long long ocol = gxo + (long long)gyo * g.sy;
    // the plane loop is uniform over the block (bounds through readfirstlane, so that the
    // compiler keeps its counter and every per-plane index in scalar registers)
    const int zm0 = __builtin_amdgcn_readfirstlane(zfirst), zm1 = __builtin_amdgcn_readfirstlane(ze - 1 + LAG);
    for (int zm = zm0; zm <= zm1; ++zm) {
        fetch_pv(zm + 2);  // in flight during the moment pass
        // u^{n-1} of this thread's output node, requested before the moment pass too
        const int zo = zm - LAG;
        const bool oin = zo >= zs && zo < ze && col_ok;
        const long long oidx = oin ? ocol + (long long)zo * sz : 0;
        const T uq0 = up0[oidx], uq1 = up1[oidx], uq2 = up2[oidx];
        int zw = zm;
        const bool zin = wrapc(zw, nz, g.per[2]);
        {   // own column first, then one pass over the halo ring
            T m[10];
            const int lx = ox + 2, ly = oy + 2;
            if (zin) moments(zm, lx, ly, m);
            else
#pragma unroll
                for (int c = 0; c < 10; ++c) m[c] = T(0);
            if constexpr (PZ) {
                own5[0] = m[4];
                own5[1] = m[5];
                own5[2] = m[7];
                own5[3] = m[8];
                own5[4] = m[9];
                zr[2][0] = m[8];
                zr[2][1] = m[9];
                zr[2][2] = m[6];
            } else {
#pragma unroll
                for (int c = 0; c < 6; ++c) s_plane<T, PZ>(ss, c, zm)[ly * MX + lx] = m[4 + c];
            }
            ru[2][0] = m[0];
            ru[2][1] = m[1];
            ru[2][2] = m[2];
            ru[2][3] = m[3];
            if (tid < NH) {
                int hx, hy;
                const int h = tid;
                if (h < 2 * MX) {
                    hy = h / MX;
                    hx = h % MX;
                } else if (h < 4 * MX) {
                    hy = TY + 2 + (h - 2 * MX) / MX;
                    hx = (h - 2 * MX) % MX;
                } else {
                    const int hh = h - 4 * MX;
                    hy = 2 + hh / 4;
                    const int sd = hh % 4;
                    hx = sd < 2 ? sd : TX + sd;
                }
                if (zin) moments(zm, hx, hy, m);
                else
#pragma unroll
                    for (int c = 0; c < 10; ++c) m[c] = T(0);
                if constexpr (PZ) {
                    halo5[0] = m[4];
                    halo5[1] = m[5];
                    halo5[2] = m[7];
                    halo5[3] = m[8];
                    halo5[4] = m[9];
                    hidx = hy * MX + hx;
                } else {
#pragma unroll
                    for (int c = 0; c < 6; ++c) s_plane<T, PZ>(ss, c, zm)[hy * MX + hx] = m[4 + c];
                }
            }
        }
        __syncthreads();
        commit_pv(zm + 2);  // replaces plane zm - 1, no longer read
        if (oin) {
            const long long idx = oidx;
            const int c0 = (oy + 2) * MX + (ox + 2);
            const T rt = ru[2 - LAG][0];
            const T ut[3] = {ru[2 - LAG][1], ru[2 - LAG][2], ru[2 - LAG][3]};
            const T sxx = s_plane<T, PZ>(ss, 0, zo)[c0], syy = s_plane<T, PZ>(ss, 1, zo)[c0];
            const T szz = PZ ? zr[1][2] : s_plane<T, PZ>(ss, 2, zo)[c0], sxy = s_plane<T, PZ>(ss, 3, zo)[c0];
            const T sxz = s_plane<T, PZ>(ss, 4, zo)[c0], syz = s_plane<T, PZ>(ss, 5, zo)[c0];
            const T u[3] = {uq0, uq1, uq2};
            T v[3];
            v[0] = T(3) * ut[0] + T(9) * (sxx * u[0] + sxy * u[1] + sxz * u[2]) - T(3) * rt * u[0];
            v[1] = T(3) * ut[1] + T(9) * (sxy * u[0] + syy * u[1] + syz * u[2]) - T(3) * rt * u[1];
            v[2] = T(3) * ut[2] + T(9) * (sxz * u[0] + syz * u[1] + szz * u[2]) - T(3) * rt * u[2];
            // V_a += 2A sum_b D_b^T s~_ab; component index of s~_ab in the ring
            constexpr int sidx[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
#pragma unroll
            for (int aa = 0; aa < 3; ++aa) {
                T f[5];
                const int cx_ = sidx[aa][0], cy_ = sidx[aa][1], cz_ = sidx[aa][2];
                const T *px = s_plane<T, PZ>(ss, cx_, zo), *py = s_plane<T, PZ>(ss, cy_, zo);
                if (xcen) {
                    v[aa] += A2 * (T(0.5) * (px[c0 - 1] - px[c0 + 1]));
                } else {
                    T d = T(0);
#pragma unroll
                    for (int o = 0; o < 5; ++o) d += dcx[o] * px[c0 + o - 2];
                    v[aa] += A2 * d;
                }
                if (ycen) {
                    v[aa] += A2 * (T(0.5) * (py[c0 - MX] - py[c0 + MX]));
                } else {
                    T d = T(0);
#pragma unroll
                    for (int o = 0; o < 5; ++o) d += dcy[o] * py[c0 + (o - 2) * MX];
                    v[aa] += A2 * d;
                }
                if constexpr (PZ) {  // periodic z: the central difference of planes zo -+ 1 (registers)
                    const int kz = cz_ == 4 ? 0 : (cz_ == 5 ? 1 : 2);
                    f[0] = f[2] = f[4] = T(0);
                    f[1] = zr[0][kz];
                    f[3] = zr[2][kz];
                } else {
#pragma unroll
                    for (int o = 0; o < 5; ++o) f[o] = s_plane<T, PZ>(ss, cz_, zo + o - 2)[c0];
                }
                v[aa] += A2 * deriv_T3(f, zo, nz, g.per[2]);
            }
            pout[idx] = rt;
            vout0[idx] = v[0];
            vout1[idx] = v[1];
            vout2[idx] = v[2];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ru[0][c] = ru[1][c];
            ru[1][c] = ru[2][c];
        }
        __syncthreads();
        if constexpr (PZ) {  // every output of plane zm - 1 is read: store plane zm (read after the next barrier)
            const int lx = ox + 2, ly = oy + 2;
#pragma unroll
            for (int c = 0; c < 5; ++c) ss[c * MP + ly * MX + lx] = own5[c];
            if (tid < NH)
#pragma unroll
                for (int c = 0; c < 5; ++c) ss[c * MP + hidx] = halo5[c];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                zr[0][c] = zr[1][c];
                zr[1][c] = zr[2][c];
            }
        }
    }
}

// PZ: every job of the launch is periodic in z (the smaller LDS layout; dynamic LDS sized to it).
// One kernel per layout, so each gets its own register allocation.
template <typename T, int Q, bool PZ>
__global__ __launch_bounds__(Tile3<T>::TX * Tile3<T>::TY) void k_adj3d_main_batch(const AdjArgs<T> *__restrict__ args,
                                                                                 const long long *__restrict__ tile0,
                                                                                 int njobs) {
    extern __shared__ __align__(16) unsigned char adj3_lds[];
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of3(tile0, njobs, b));
    const AdjArgs<T> &a = args[j];
    int bx, by, bz;
    tile_coords3<T>(a.g, a.g.zca, njobs == 1 ? b : b - tile0[j], bx, by, bz);
    adj3d_main_body<T, Q, PZ>(a, bx, by, bz, reinterpret_cast<T *>(adj3_lds));
}

long long fwd_blocks3d(const Geom &g, int lattice, int esz) {
    (void)lattice;
    const int TX = esz == 8 ? Tile3<double>::TX : Tile3<float>::TX;
    const int TY = esz == 8 ? Tile3<double>::TY : Tile3<float>::TY;
    return (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) * ((g.n[2] + g.zc - 1) / g.zc);
}

// z planes marched per block: the longest chunk (Tile3::ZC) while the grid still yields about
// one block per slot of the chip (256 CUs x 4); halved, down to 8 planes, for smaller grids, where
// a launch would otherwise last as long as one block's march (a block also loads and evaluates
// 2-4 planes beyond its chunk, which is why the floor is not lower); then evened out over the
// chunks of nz.  Measured on the served mix (3D jobs 64^3..160^3 get 8 planes): 3.0 -> 3.35
// evals/s batched, 2.4 -> 3.25 one job at a time; 256^3 keeps 32 (16 was slower there).
int choose_zc3(const Geom &g, int esz) {
    constexpr long long kTargetBlocks = 1024;
    constexpr int kMinPlanes = 8;
    const int TX = esz == 8 ? Tile3<double>::TX : Tile3<float>::TX;
    const int TY = esz == 8 ? Tile3<double>::TY : Tile3<float>::TY;
    const long long cols = (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY);
    int zc = esz == 8 ? Tile3<double>::ZC : Tile3<float>::ZC;
    while (zc > kMinPlanes && cols * ((g.n[2] + zc - 1) / zc) < kTargetBlocks) zc /= 2;
    const int nch = (g.n[2] + zc - 1) / zc;
    return (g.n[2] + nch - 1) / nch;
}

long long tiles3d(const Geom &g, int esz) { return fwd_blocks3d(g, 0, esz); }

long long tiles3d_adj(const Geom &g, int esz) {
    const int TX = esz == 8 ? Tile3<double>::TX : Tile3<float>::TX;
    const int TY = esz == 8 ? Tile3<double>::TY : Tile3<float>::TY;
    return (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) * ((g.n[2] + g.zca - 1) / g.zca);
}

// z planes per block of the z-marching adjoint.  Its LDS admits four FP32 blocks per CU when the
// domain is periodic in z (1024 slots), else two.  Where the forward keeps its longest chunk (a
// large grid), the adjoint takes the number
// of chunks (at most the forward's) that minimises rounds x (planes + 3): the blocks of a round
// run together, and a block marches about 3 planes beyond its chunk.  On 256^3 this picks 64
// planes (1024 blocks, one round).  With three blocks per CU the measured launch times followed
// the model's order (86 planes 469 us, 43 planes 477, 29 planes 489, 32 planes 506).  Elsewhere,
// and in FP64, the forward's chunk.
int choose_zca3(const Geom &g, int esz) {
    const long long kAdjSlots = g.per[2] ? 1024 : 512;
    if (esz != 4 || g.zc < Tile3<float>::ZC) return g.zc;
    const long long cols = (long long)((g.n[0] + Tile3<float>::TX - 1) / Tile3<float>::TX) *
                           ((g.n[1] + Tile3<float>::TY - 1) / Tile3<float>::TY);
    const int nz = g.n[2], nchf = (nz + g.zc - 1) / g.zc;
    int best = nchf;
    long long bestc = -1;
    for (int nch = 1; nch <= nchf; ++nch) {
        const long long rounds = (cols * nch + kAdjSlots - 1) / kAdjSlots;
        const long long cost = rounds * ((nz + nch - 1) / nch + 3);
        if (bestc < 0 || cost < bestc) {
            bestc = cost;
            best = nch;
        }
    }
    return (nz + best - 1) / best;
}

long long xfer_blocks3d(long long cells, int esz) {
    const long long nt = esz == 8 ? Tile3<double>::TX * Tile3<double>::TY : Tile3<float>::TX * Tile3<float>::TY;
    return (cells + nt - 1) / nt;
}

template <typename T>
hipError_t launch_fwd3d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, int lattice, bool pz, hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    const dim3 blk(Tile3<T>::TX * Tile3<T>::TY);
    const dim3 grid((unsigned)ntiles);
    const unsigned lds19 = (unsigned)Fwd3Lds<T, 19>::bytes(pz), lds15 = (unsigned)Fwd3Lds<T, 15>::bytes(pz);
    if (lattice == 2 && pz) hipLaunchKernelGGL((k_fwd3d_batch<T, 19, true>), grid, blk, lds19, s, args, tile0, njobs);
    else if (lattice == 2) hipLaunchKernelGGL((k_fwd3d_batch<T, 19, false>), grid, blk, lds19, s, args, tile0, njobs);
    else if (pz) hipLaunchKernelGGL((k_fwd3d_batch<T, 15, true>), grid, blk, lds15, s, args, tile0, njobs);
    else hipLaunchKernelGGL((k_fwd3d_batch<T, 15, false>), grid, blk, lds15, s, args, tile0, njobs);
    return hipGetLastError();
}

// Transfer blocks alone, without the stencil's LDS: used where the transfer of the next step
// runs beside launches of another stream (segment recompute during the reverse sweep) or with
// no stencil at all, so that its many short blocks hold no LDS.
template <typename T>
__global__ __launch_bounds__(Tile3<T>::TX * Tile3<T>::TY) void k_xfer3d_batch(const FwdArgs<T> *__restrict__ args,
                                                                            const long long *__restrict__ tile0,
                                                                            int njobs) {
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of3(tile0, njobs, b));
    const FwdArgs<T> &a = args[j];
    const long long t = njobs == 1 ? b : b - tile0[j];
    transfer_box<T, 3, Tile3<T>::TX * Tile3<T>::TY>(a.des, a.mnext, a.box, a.knext, a.usnext, t);
}

template <typename T>
hipError_t launch_xfer3d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs, long long ntiles,
                               hipStream_t s) {
    if (njobs == 0 || ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_xfer3d_batch<T>, dim3((unsigned)ntiles), dim3(Tile3<T>::TX * Tile3<T>::TY), 0, s,
                       args, tile0, njobs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj3d_batch(const AdjArgs<T> *args, const long long *blk0, long long nblk,
                              const long long *tile0, long long ntiles, int njobs, int lattice, bool pz,
                              hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj3d_prep_batch<T>, dim3((unsigned)nblk), dim3(kBlock), 0, s, args, blk0, njobs);
    const dim3 blk(Tile3<T>::TX * Tile3<T>::TY);
    const unsigned lds = (unsigned)Adj3Lds<T>::bytes(pz);
    const dim3 grid((unsigned)ntiles);
    if (lattice == 2 && pz) hipLaunchKernelGGL((k_adj3d_main_batch<T, 19, true>), grid, blk, lds, s, args, tile0, njobs);
    else if (lattice == 2) hipLaunchKernelGGL((k_adj3d_main_batch<T, 19, false>), grid, blk, lds, s, args, tile0, njobs);
    else if (pz) hipLaunchKernelGGL((k_adj3d_main_batch<T, 15, true>), grid, blk, lds, s, args, tile0, njobs);
    else hipLaunchKernelGGL((k_adj3d_main_batch<T, 15, false>), grid, blk, lds, s, args, tile0, njobs);
    return hipGetLastError();
}

#define LKS_INST3(T)                                                                                  \
    template hipError_t launch_fwd3d_batch<T>(const FwdArgs<T> *, const long long *, int, long long,  \
                                              int, bool, hipStream_t);                                \
    template hipError_t launch_adj3d_batch<T>(const AdjArgs<T> *, const long long *, long long,       \
                                              const long long *, long long, int, int, bool, hipStream_t); \
    template hipError_t launch_xfer3d_batch<T>(const FwdArgs<T> *, const long long *, int, long long,   \
                                               hipStream_t);
LKS_INST3(float)
LKS_INST3(double)
#undef LKS_INST3

}  // namespace lks

// 3D kernels (D3Q19 and D3Q15).
//
// Forward step, marching along z (Algorithm 1 body, Sec. 2.2-2.3): a block owns a TX x TY column
// of output nodes and a chunk of ZC planes.  Velocity planes z-2 .. z+2 (x-y halo 2) sit in an
// LDS ring; the equilibrium E_i of plane z (x-y halo 1) is evaluated once into LDS; each thread
// then adds the E_i pulled by its own column into three in-flight output planes held in
// registers (c_z = -1 completes plane z-1, c_z = 0 feeds plane z, c_z = +1 plane z+1), and
// finishes plane z-1: transfer gather, VPM update, composite boundary rules, objective partial.
// The next velocity plane is fetched into registers before the stencil work of the current one.
//
// Adjoint step in two kernels.  The first is pointwise: lambda = Lambda^n + dj^n/dX^n, the
// boundary transpose (seeds of face nodes returned to the interior node they copy from), the
// force transpose V* = V / (1 + kappa + kappa_s) and kappa_bar on the footprint box.  The second
// marches along z: (P*, V*) planes (halo 3) in an LDS ring, the pull transpose and its w-weighted
// moments rho~, u~, s~ per plane (halo 2; a ring of five s~ planes), and Lambda^{n-1} of the
// plane two behind from the transposed equilibrium and the transposed strain operator.
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
template <>
struct Tile3<float> {
    static constexpr int TX = 32, TY = 8, ZC = 32;
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
template <typename T, int Q>
__device__ __forceinline__ void fwd3d_body(const FwdArgs<T> &a, int bx, int by, int bz, long long blin) {
    constexpr int TX = Tile3<T>::TX, TY = Tile3<T>::TY, ZC = Tile3<T>::ZC, NT = TX * TY;
    constexpr int UX = TX + 4, UY = TY + 4, UP = UX * UY;  // velocity plane, halo 2
    constexpr int EX = TX + 2, EY = TY + 2, EP = EX * EY;  // E_i plane, halo 1
    constexpr int NU = (UP + NT - 1) / NT, NR = (EP + NT - 1) / NT;
    __shared__ T su[5][3][UP];
    __shared__ T sE[Q][EP];
    __shared__ double sh[NT / 64];

    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY, zs = bz * ZC;
    const int ze = min(zs + ZC, nz);
    const int ox = tid % TX, oy = tid / TX;
    const T A = a.A;

    T ureg[NU][3];
    T rreg[NR];
    auto fetch_u = [&](int zp) {
        int zw = zp;
        const bool zin = wrapc(zw, nz, g.per[2]);
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            const int i = tid + k * NT;
            ureg[k][0] = ureg[k][1] = ureg[k][2] = T(0);
            if (i >= UP || !zin) continue;
            int gx = x0 - 2 + i % UX, gy = y0 - 2 + i / UX;
            if (!wrapc(gx, nx, g.per[0]) || !wrapc(gy, ny, g.per[1])) continue;
            const long long idx = gx + gy * g.sy + zw * g.sz;
            ureg[k][0] = a.uin[0][idx];
            ureg[k][1] = a.uin[1][idx];
            ureg[k][2] = a.uin[2][idx];
        }
    };
    auto commit_u = [&](int zp) {
        const int sl = ring5(zp);
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
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int i = tid + k * NT;
            rreg[k] = T(0);
            if (i >= EP || !zin) continue;
            int gx = x0 - 1 + i % EX, gy = y0 - 1 + i / EX;
            if (!wrapc(gx, nx, g.per[0]) || !wrapc(gy, ny, g.per[1])) continue;
            rreg[k] = a.rin[gx + gy * g.sy + zw * g.sz];
        }
    };

    for (int zp = zs - 3; zp <= zs + 1; ++zp) {
        fetch_u(zp);
        commit_u(zp);
    }
    fetch_r(zs - 1);
    __syncthreads();

    T acc[3][4];
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[t][0] = acc[t][1] = acc[t][2] = acc[t][3] = T(0);
    double jacc = 0.0;
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;

    for (int zc = zs - 1; zc <= ze; ++zc) {
        T rcur[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) rcur[k] = rreg[k];
        fetch_u(zc + 3);  // in flight during the stencil work below
        fetch_r(zc + 1);
        int zw = zc;
        const bool zin = wrapc(zw, nz, g.per[2]);
        if (zin) {
            const int s0 = ring5(zc), sm1 = ring5(zc - 1), sp1 = ring5(zc + 1), sm2 = ring5(zc - 2),
                      sp2 = ring5(zc + 2);
#pragma unroll
            for (int k = 0; k < NR; ++k) {
                const int i = tid + k * NT;
                if (i >= EP) continue;
                const int lx = i % EX, ly = i / EX;
                const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
                if (!g.per[0] && (gx < 0 || gx >= nx)) continue;
                if (!g.per[1] && (gy < 0 || gy >= ny)) continue;
                const int c0 = (ly + 1) * UX + (lx + 1);
                T u[3], du[3][3];  // du[c][b] = d u_c / d x_b
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const T *p = su[s0][c];
                    u[c] = p[c0];
                    du[c][0] = dcoord(c0 >= 2 ? p[c0 - 2] : T(0), p[c0 - 1], p[c0], p[c0 + 1],
                                      p[c0 + 2], gx, nx, g.per[0]);
                    du[c][1] = dcoord(ly + 1 >= 2 ? p[c0 - 2 * UX] : T(0), p[c0 - UX], p[c0],
                                      p[c0 + UX], ly + 3 < UY ? p[c0 + 2 * UX] : T(0), gy, ny,
                                      g.per[1]);
                    du[c][2] = dcoord(su[sm2][c][c0], su[sm1][c][c0], p[c0], su[sp1][c][c0],
                                      su[sp2][c][c0], zw, nz, g.per[2]);
                }
                const T r = rcur[k];
                const T a0 = r - T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                T tt[3][3];
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q)
                        tt[p][q] = T(4.5) * u[p] * u[q] + A * (du[p][q] + du[q][p]);
#pragma unroll
                for (int q = 0; q < Q; ++q) {
                    constexpr int dummy = 0;
                    (void)dummy;
                    const int cx = cq<Q>(q, 0), cy = cq<Q>(q, 1), cz = cq<Q>(q, 2);
                    T v = a0 + T(3) * (T(cx) * u[0] + T(cy) * u[1] + T(cz) * u[2]);
                    v += T(cx * cx) * tt[0][0] + T(cy * cy) * tt[1][1] + T(cz * cz) * tt[2][2];
                    v += T(2 * cx * cy) * tt[0][1] + T(2 * cx * cz) * tt[0][2] + T(2 * cy * cz) * tt[1][2];
                    sE[q][i] = T(wq<Q>(q)) * v;
                }
            }
        }
        __syncthreads();
        commit_u(zc + 3);
        // pull: output (x, y, zo) takes E_i from (x - cx, y - cy) in plane zo - cz
        if (zin) {
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                const int cx = cq<Q>(q, 0), cy = cq<Q>(q, 1), cz = cq<Q>(q, 2);
                const T e = sE[q][(oy + 1 - cy) * EX + (ox + 1 - cx)];
                const int t = cz + 1;  // cz = -1 -> plane zc - 1, 0 -> zc, +1 -> zc + 1
                acc[t][0] += e;
                acc[t][1] += T(cx) * e;
                acc[t][2] += T(cy) * e;
                acc[t][3] += T(cz) * e;
            }
        }
        const int zo = zc - 1;
        const int gx = x0 + ox, gy = y0 + oy;
        if (zo >= zs && zo < ze && gx < nx && gy < ny && !on_face(g, 0, gx) && !on_face(g, 1, gy) &&
            !on_face(g, 2, zo)) {
            const T rs = acc[0][0];
            T kap = 0, us[3] = {0, 0, 0};
            if (in_box(a.m, 3, gx, gy, zo)) {
                const long long bi = box_index(a.box, a.m, 3, gx, gy, zo);
                kap = a.kin[bi];
                us[0] = a.usin[0][bi];
                us[1] = a.usin[1][bi];
                us[2] = a.usin[2][bi];
            }
            const long long idx = gx + gy * g.sy + zo * g.sz;
            const T ks = a.kstatic ? a.kstatic[idx] : T(0);
            const T inv = T(1) / (T(1) + kap + ks);
            T nu[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) nu[c] = (acc[0][1 + c] + kap * us[c] + a.gf[c]) * inv;
            a.rout[idx] = rs;
            a.uout[0][idx] = nu[0];
            a.uout[1][idx] = nu[1];
            a.uout[2][idx] = nu[2];
            if (obj_on && (!a.obj.mask || a.obj.mask[idx]))
                jacc += obj_density<T>(a.obj, gx, gy, zo, (double)rs, nu, kap, us);
            const int c3[3] = {gx, gy, zo};
            const T v[4] = {rs, nu[0], nu[1], nu[2]};
            push_boundary<T, 3>(g, a.bc, c3, v, [&](const int p[3], const T pv[4]) {
                const long long pi = p[0] + p[1] * g.sy + p[2] * g.sz;
                a.rout[pi] = pv[0];
                a.uout[0][pi] = pv[1];
                a.uout[1][pi] = pv[2];
                a.uout[2][pi] = pv[3];
                if (obj_on && (!a.obj.mask || a.obj.mask[pi])) {
                    const T pu[3] = {pv[1], pv[2], pv[3]}, z3[3] = {0, 0, 0};
                    jacc += obj_density<T>(a.obj, p[0], p[1], p[2], (double)pv[0], pu, T(0), z3);
                }
            });
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            acc[0][c] = acc[1][c];
            acc[1][c] = acc[2][c];
            acc[2][c] = T(0);
        }
        __syncthreads();
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

template <typename T>
__device__ __forceinline__ void tile_coords3(const Geom &g, long long t, int &bx, int &by, int &bz) {
    const int nbx = (g.n[0] + Tile3<T>::TX - 1) / Tile3<T>::TX;
    const int nby = (g.n[1] + Tile3<T>::TY - 1) / Tile3<T>::TY;
    bx = (int)(t % nbx);
    by = (int)((t / nbx) % nby);
    bz = (int)(t / ((long long)nbx * nby));
}

template <typename T>
__device__ __forceinline__ long long stencil_tiles3(const Geom &g) {
    return (long long)((g.n[0] + Tile3<T>::TX - 1) / Tile3<T>::TX) *
           ((g.n[1] + Tile3<T>::TY - 1) / Tile3<T>::TY) * ((g.n[2] + Tile3<T>::ZC - 1) / Tile3<T>::ZC);
}

template <typename T, int Q>
__global__ __launch_bounds__(Tile3<T>::TX * Tile3<T>::TY) void k_fwd3d_batch(const FwdArgs<T> *args,
                                                                            const long long *tile0,
                                                                            int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of3(tile0, njobs, b);
    const FwdArgs<T> &a = args[j];
    const long long t = njobs == 1 ? b : b - tile0[j];  // one job: tile0 = {0}
    const long long ns = (a.mode & FWD_STENCIL) ? stencil_tiles3<T>(a.g) : 0;
    if (t >= ns) {  // extra blocks: transfer of the next step onto its footprint box
        transfer_box<T, 3, Tile3<T>::TX * Tile3<T>::TY>(a.des, a.mnext, a.box, a.knext, a.usnext, t - ns);
        return;
    }
    int bx, by, bz;
    tile_coords3<T>(a.g, t, bx, by, bz);
    fwd3d_body<T, Q>(a, bx, by, bz, t);
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

template <typename T>
__device__ __forceinline__ void adj3d_prep_body(const AdjArgs<T> &a, long long blk) {
    const Geom &g = a.g;
    const long long ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    const long long t = blk * kBlock + threadIdx.x;
    if (t >= ncell) return;
    const int x = (int)(t % g.n[0]);
    const int y = (int)((t / g.n[0]) % g.n[1]);
    const int z = (int)(t / ((long long)g.n[0] * g.n[1]));
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj3d_prep_batch(const AdjArgs<T> *args,
                                                             const long long *blk0, int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of3(blk0, njobs, b);
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

template <typename T, int Q>
__device__ __forceinline__ void adj3d_main_body(const AdjArgs<T> &a, int bx, int by, int bz) {
    constexpr int TX = Tile3<T>::TX, TY = Tile3<T>::TY, ZC = Tile3<T>::ZC, NT = TX * TY;
    constexpr int PX = TX + 6, PY = TY + 6, PP = PX * PY;  // (P*, V*) plane, halo 3
    constexpr int MX = TX + 4, MY = TY + 4, MP = MX * MY;  // moment plane, halo 2
    constexpr int NP = (PP + NT - 1) / NT;
    constexpr int NH = MP - NT;                            // halo moment nodes
    static_assert(NH <= NT, "one halo pass");
    __shared__ T spv[3][4][PP];
    __shared__ T ss[5][6][MP];  // s~ xx, yy, zz, xy, xz, yz

    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY, zs = bz * ZC;
    const int ze = min(zs + ZC, nz);
    const int ox = tid % TX, oy = tid / TX;

    T preg[NP][4];
    auto fetch_pv = [&](int zp) {
        int zw = zp;
        const bool zin = wrapc(zw, nz, g.per[2]);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const int i = tid + k * NT;
            preg[k][0] = preg[k][1] = preg[k][2] = preg[k][3] = T(0);
            if (i >= PP || !zin) continue;
            int gx = x0 - 3 + i % PX, gy = y0 - 3 + i / PX;
            if (!wrapc(gx, nx, g.per[0]) || !wrapc(gy, ny, g.per[1])) continue;
            const long long idx = gx + gy * g.sy + zw * g.sz;
            preg[k][0] = a.Ps[idx];
            preg[k][1] = a.Vs[0][idx];
            preg[k][2] = a.Vs[1][idx];
            preg[k][3] = a.Vs[2][idx];
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
    // moments of the pull transpose at moment-plane node (lx, ly) of plane zm
    auto moments = [&](int zm, int lx, int ly, T m[10]) {
#pragma unroll
        for (int c = 0; c < 10; ++c) m[c] = T(0);
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int cx = cq<Q>(q, 0), cy = cq<Q>(q, 1), cz = cq<Q>(q, 2);
            const int sl = ring3(zm + cz);
            const int pi = (ly + 1 + cy) * PX + (lx + 1 + cx);
            const T eb = spv[sl][0][pi] + T(cx) * spv[sl][1][pi] + T(cy) * spv[sl][2][pi] +
                         T(cz) * spv[sl][3][pi];
            const T we = T(wq<Q>(q)) * eb;
            m[0] += we;                // rho~
            m[1] += T(cx) * we;        // u~
            m[2] += T(cy) * we;
            m[3] += T(cz) * we;
            m[4] += T(cx * cx) * we;   // s~ xx, yy, zz, xy, xz, yz
            m[5] += T(cy * cy) * we;
            m[6] += T(cz * cz) * we;
            m[7] += T(cx * cy) * we;
            m[8] += T(cx * cz) * we;
            m[9] += T(cy * cz) * we;
        }
    };

    for (int zp = zs - 3; zp <= zs - 1; ++zp) {
        fetch_pv(zp);
        commit_pv(zp);
    }
    __syncthreads();
    T ru[3][4];  // rho~, u~ of the own column for planes zm-2, zm-1, zm
#pragma unroll
    for (int t = 0; t < 3; ++t) ru[t][0] = ru[t][1] = ru[t][2] = ru[t][3] = T(0);
    const T A2 = T(2) * a.A;

    for (int zm = zs - 2; zm <= ze + 1; ++zm) {
        fetch_pv(zm + 2);  // in flight during the moment pass
        int zw = zm;
        const bool zin = wrapc(zw, nz, g.per[2]);
        const int sm = ring5(zm);
        {   // own column first, then one pass over the halo ring
            T m[10];
            const int lx = ox + 2, ly = oy + 2;
            if (zin) moments(zm, lx, ly, m);
            else
#pragma unroll
                for (int c = 0; c < 10; ++c) m[c] = T(0);
#pragma unroll
            for (int c = 0; c < 6; ++c) ss[sm][c][ly * MX + lx] = m[4 + c];
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
#pragma unroll
                for (int c = 0; c < 6; ++c) ss[sm][c][hy * MX + hx] = m[4 + c];
            }
        }
        __syncthreads();
        commit_pv(zm + 2);  // replaces plane zm - 1, no longer read
        const int zo = zm - 2;
        const int gx = x0 + ox, gy = y0 + oy;
        if (zo >= zs && zo < ze && gx < nx && gy < ny) {
            const long long idx = gx + gy * g.sy + zo * g.sz;
            const int c0 = (oy + 2) * MX + (ox + 2);
            const int so = ring5(zo);
            const T rt = ru[0][0];
            const T ut[3] = {ru[0][1], ru[0][2], ru[0][3]};
            const T sxx = ss[so][0][c0], syy = ss[so][1][c0], szz = ss[so][2][c0];
            const T sxy = ss[so][3][c0], sxz = ss[so][4][c0], syz = ss[so][5][c0];
            const T u[3] = {a.uprev[0][idx], a.uprev[1][idx], a.uprev[2][idx]};
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
#pragma unroll
                for (int o = 0; o < 5; ++o) f[o] = ss[so][cx_][c0 + o - 2];
                v[aa] += A2 * deriv_T3(f, gx, nx, g.per[0]);
#pragma unroll
                for (int o = 0; o < 5; ++o) f[o] = ss[so][cy_][c0 + (o - 2) * MX];
                v[aa] += A2 * deriv_T3(f, gy, ny, g.per[1]);
#pragma unroll
                for (int o = 0; o < 5; ++o) f[o] = ss[ring5(zo + o - 2)][cz_][c0];
                v[aa] += A2 * deriv_T3(f, zo, nz, g.per[2]);
            }
            a.Pout[idx] = rt;
            a.Vout[0][idx] = v[0];
            a.Vout[1][idx] = v[1];
            a.Vout[2][idx] = v[2];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            ru[0][c] = ru[1][c];
            ru[1][c] = ru[2][c];
        }
        __syncthreads();
    }
}

template <typename T, int Q>
__global__ __launch_bounds__(Tile3<T>::TX * Tile3<T>::TY) void k_adj3d_main_batch(const AdjArgs<T> *args,
                                                                                 const long long *tile0,
                                                                                 int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of3(tile0, njobs, b);
    const AdjArgs<T> &a = args[j];
    int bx, by, bz;
    tile_coords3<T>(a.g, njobs == 1 ? b : b - tile0[j], bx, by, bz);
    adj3d_main_body<T, Q>(a, bx, by, bz);
}

long long fwd_blocks3d(const Geom &g, int lattice, int esz) {
    (void)lattice;
    const int TX = esz == 8 ? Tile3<double>::TX : Tile3<float>::TX;
    const int TY = esz == 8 ? Tile3<double>::TY : Tile3<float>::TY;
    const int ZC = esz == 8 ? Tile3<double>::ZC : Tile3<float>::ZC;
    return (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) * ((g.n[2] + ZC - 1) / ZC);
}

long long tiles3d(const Geom &g, int esz) { return fwd_blocks3d(g, 0, esz); }

long long xfer_blocks3d(long long cells, int esz) {
    const long long nt = esz == 8 ? Tile3<double>::TX * Tile3<double>::TY : Tile3<float>::TX * Tile3<float>::TY;
    return (cells + nt - 1) / nt;
}

template <typename T>
hipError_t launch_fwd3d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, int lattice, hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    const dim3 blk(Tile3<T>::TX * Tile3<T>::TY);
    if (lattice == 2) hipLaunchKernelGGL((k_fwd3d_batch<T, 19>), dim3((unsigned)ntiles), blk, 0, s, args, tile0, njobs);
    else hipLaunchKernelGGL((k_fwd3d_batch<T, 15>), dim3((unsigned)ntiles), blk, 0, s, args, tile0, njobs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj3d_batch(const AdjArgs<T> *args, const long long *blk0, long long nblk,
                              const long long *tile0, long long ntiles, int njobs, int lattice,
                              hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj3d_prep_batch<T>, dim3((unsigned)nblk), dim3(kBlock), 0, s, args, blk0, njobs);
    const dim3 blk(Tile3<T>::TX * Tile3<T>::TY);
    if (lattice == 2) hipLaunchKernelGGL((k_adj3d_main_batch<T, 19>), dim3((unsigned)ntiles), blk, 0, s, args, tile0, njobs);
    else hipLaunchKernelGGL((k_adj3d_main_batch<T, 15>), dim3((unsigned)ntiles), blk, 0, s, args, tile0, njobs);
    return hipGetLastError();
}

#define LKS_INST3(T)                                                                                  \
    template hipError_t launch_fwd3d_batch<T>(const FwdArgs<T> *, const long long *, int, long long,  \
                                              int, hipStream_t);                                      \
    template hipError_t launch_adj3d_batch<T>(const AdjArgs<T> *, const long long *, long long,       \
                                              const long long *, long long, int, int, hipStream_t);
LKS_INST3(float)
LKS_INST3(double)
#undef LKS_INST3

}  // namespace lks

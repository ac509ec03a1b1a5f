// 2D D2Q9 kernels: one fused forward step and one fused adjoint step per launch.
//
// Forward step (Algorithm 1 body, Sec. 2.2-2.3), per 64x8 tile of output nodes:
//   stage u (halo 2) and rho - 1 (halo 1) in LDS; evaluate the equilibrium E_i of every node of
//   the tile plus a halo of 1 (strain from central differences, one-sided on non-periodic faces);
//   pull rho* = sum_i E_i(x - c_i), m* = sum_i c_i E_i(x - c_i); transfer kappa and u_S at the node
//   by a gather over the rotated design grid; implicit VPM update; composite boundary rules for the
//   face nodes that copy from this node; FP64 objective partial; last-block reduction.
// Adjoint step (the exact transpose, in reverse order), per 64x8 tile:
//   lambda = Lambda + dj/dX on the tile plus halo 4; boundary transpose and force transpose give
//   (P*, V*) on halo 3 and kappa_bar on the tile; the pull transpose E~_i(y) = P*(y+c_i) +
//   c_i.V*(y+c_i) and its w-weighted moments (rho~, u~, s~) on halo 2; then Lambda^{n-1} from the
//   transposed equilibrium and the transposed strain operator.
// rho is carried as rho - 1 on the GPU: the constant part adds exactly 1 to rho* and nothing to
// m* (sum_i w_i = 1, sum_i w_i c_i = 0), so the update is unchanged and FP32 keeps the fluctuation.
#include "lks_device.hpp"

namespace lks {

namespace d2q9 {
// D2Q9 velocities and weights (index 0 = rest)
constexpr double W0 = 4.0 / 9.0, WA = 1.0 / 9.0, WD = 1.0 / 36.0;
__device__ constexpr int cx(int i) {
    return i == 1 || i == 5 || i == 8 ? 1 : (i == 3 || i == 6 || i == 7 ? -1 : 0);
}
__device__ constexpr int cy(int i) {
    return i == 2 || i == 5 || i == 6 ? 1 : (i == 4 || i == 7 || i == 8 ? -1 : 0);
}
__device__ constexpr double wt(int i) { return i == 0 ? W0 : (i < 5 ? WA : WD); }
}  // namespace d2q9

constexpr int TX = 64, TY = 8;

template <typename T>
__device__ __forceinline__ void fwd2d_body(const FwdArgs<T> &a, int bx, int by, long long blin) {
    constexpr int UX = TX + 4, UY = TY + 4;  // u staged with halo 2, origin (x0-2, y0-2)
    constexpr int EX = TX + 2, EY = TY + 2;  // rho and E_i with halo 1, origin (x0-1, y0-1)
    __shared__ T su[2][UY][UX];
    __shared__ T sr[EY][EX];
    __shared__ T sE[8][EY][EX];
    __shared__ double sh4[4];

    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY;
    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1];

    for (int i = tid; i < UX * UY; i += kBlock) {
        const int lx = i % UX, ly = i / UX;
        int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        T ux = 0, uy = 0;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1])) {
            const long long idx = gx + gy * g.sy;
            ux = a.uin[0][idx];
            uy = a.uin[1][idx];
        }
        su[0][ly][lx] = ux;
        su[1][ly][lx] = uy;
    }
    for (int i = tid; i < EX * EY; i += kBlock) {
        const int lx = i % EX, ly = i / EX;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        T r = 0;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1])) r = a.rin[gx + gy * g.sy];
        sr[ly][lx] = r;
    }
    __syncthreads();

    // equilibrium of every staged node (Sec. 2.2): E_i = w_i [rho + 3 c.u + 4.5 (c.u)^2 - 1.5 u^2
    // + A c.S.c], S_ab = d_b u_a + d_a u_b; the rest direction is evaluated at the puller
    const T A = a.A;
    for (int i = tid; i < EX * EY; i += kBlock) {
        const int lx = i % EX, ly = i / EX;
        int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
        if (!g.per[0] && (gx < 0 || gx >= nx)) continue;
        if (!g.per[1] && (gy < 0 || gy >= ny)) continue;
        const int ux_ = lx + 1, uy_ = ly + 1;  // position in su
        const int cxn = gx, cyn = gy;          // true coordinate on non-periodic axes
        T dxux, dxuy, dyux, dyuy;
        if (!g.per[0] && (cxn == 0 || cxn == nx - 1)) {
            const int s = cxn == 0 ? 1 : -1;
            dxux = T(s) * (T(-1.5) * su[0][uy_][ux_] + T(2) * su[0][uy_][ux_ + s] - T(0.5) * su[0][uy_][ux_ + 2 * s]);
            dxuy = T(s) * (T(-1.5) * su[1][uy_][ux_] + T(2) * su[1][uy_][ux_ + s] - T(0.5) * su[1][uy_][ux_ + 2 * s]);
        } else {
            dxux = T(0.5) * (su[0][uy_][ux_ + 1] - su[0][uy_][ux_ - 1]);
            dxuy = T(0.5) * (su[1][uy_][ux_ + 1] - su[1][uy_][ux_ - 1]);
        }
        if (!g.per[1] && (cyn == 0 || cyn == ny - 1)) {
            const int s = cyn == 0 ? 1 : -1;
            dyux = T(s) * (T(-1.5) * su[0][uy_][ux_] + T(2) * su[0][uy_ + s][ux_] - T(0.5) * su[0][uy_ + 2 * s][ux_]);
            dyuy = T(s) * (T(-1.5) * su[1][uy_][ux_] + T(2) * su[1][uy_ + s][ux_] - T(0.5) * su[1][uy_ + 2 * s][ux_]);
        } else {
            dyux = T(0.5) * (su[0][uy_ + 1][ux_] - su[0][uy_ - 1][ux_]);
            dyuy = T(0.5) * (su[1][uy_ + 1][ux_] - su[1][uy_ - 1][ux_]);
        }
        const T ux = su[0][uy_][ux_], uy = su[1][uy_][ux_], r = sr[ly][lx];
        const T a0 = r - T(1.5) * (ux * ux + uy * uy);
        const T bx = T(3) * ux, by = T(3) * uy;
        const T txx = T(4.5) * ux * ux + A * T(2) * dxux;
        const T tyy = T(4.5) * uy * uy + A * T(2) * dyuy;
        const T txy2 = T(2) * (T(4.5) * ux * uy + A * (dyux + dxuy));
        const T wa = T(d2q9::WA), wd = T(d2q9::WD);
        sE[0][ly][lx] = wa * (a0 + bx + txx);                    // ( 1, 0)
        sE[1][ly][lx] = wa * (a0 + by + tyy);                    // ( 0, 1)
        sE[2][ly][lx] = wa * (a0 - bx + txx);                    // (-1, 0)
        sE[3][ly][lx] = wa * (a0 - by + tyy);                    // ( 0,-1)
        sE[4][ly][lx] = wd * (a0 + bx + by + txx + tyy + txy2);  // ( 1, 1)
        sE[5][ly][lx] = wd * (a0 - bx + by + txx + tyy - txy2);  // (-1, 1)
        sE[6][ly][lx] = wd * (a0 - bx - by + txx + tyy + txy2);  // (-1,-1)
        sE[7][ly][lx] = wd * (a0 + bx - by + txx + tyy - txy2);  // ( 1,-1)
    }
    __syncthreads();

    double jacc = 0.0;
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    for (int k = 0; k < (TX * TY) / kBlock; ++k) {
        const int lx = tid % TX, ly = tid / TX + k * (kBlock / TX);
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        if (on_face(g, 0, gx) || on_face(g, 1, gy)) continue;  // written by push_boundary
        const int ex = lx + 1, ey = ly + 1;
        const T ux = su[0][ly + 2][lx + 2], uy = su[1][ly + 2][lx + 2], r = sr[ey][ex];
        const T e0 = T(d2q9::W0) * (r - T(1.5) * (ux * ux + uy * uy));
        // pull from x - c_i
        const T e1 = sE[0][ey][ex - 1], e2 = sE[1][ey - 1][ex], e3 = sE[2][ey][ex + 1],
                e4 = sE[3][ey + 1][ex], e5 = sE[4][ey - 1][ex - 1], e6 = sE[5][ey - 1][ex + 1],
                e7 = sE[6][ey + 1][ex + 1], e8 = sE[7][ey + 1][ex - 1];
        const T rs = e0 + (e1 + e2 + e3 + e4) + (e5 + e6 + e7 + e8);
        const T mx = (e1 - e3) + (e5 - e6) + (e8 - e7);
        const T my = (e2 - e4) + (e5 + e6) - (e7 + e8);
        T kap = 0, us[3] = {0, 0, 0};
        const bool inb = in_box(a.m, 2, gx, gy, 0);
        if (inb) gather_kappa<T, 2>(a.des, a.m, gx, gy, 0, kap, us);
        const long long idx = gx + gy * g.sy;
        const T ks = a.kstatic ? a.kstatic[idx] : T(0);
        const T inv = T(1) / (T(1) + kap + ks);
        const T nux = (mx + kap * us[0] + a.gf[0]) * inv;
        const T nuy = (my + kap * us[1] + a.gf[1]) * inv;
        a.rout[idx] = rs;
        a.uout[0][idx] = nux;
        a.uout[1][idx] = nuy;
        if (a.kbox && inb) {
            const long long bi = box_index(a.box, a.m, 2, gx, gy, 0);
            a.kbox[bi] = kap;
            a.usbox[0][bi] = us[0];
            a.usbox[1][bi] = us[1];
        }
        const T uv[3] = {nux, nuy, T(0)};
        if (obj_on && (!a.obj.mask || a.obj.mask[idx]))
            jacc += obj_density<T>(a.obj, gx, gy, 0, (double)rs, uv, kap, us);
        const int c[3] = {gx, gy, 0};
        const T v[4] = {rs, nux, nuy, T(0)};
        push_boundary<T, 2>(g, a.bc, c, v, [&](const int p[3], const T pv[4]) {
            const long long pi = p[0] + p[1] * g.sy;
            a.rout[pi] = pv[0];
            a.uout[0][pi] = pv[1];
            a.uout[1][pi] = pv[2];
            if (obj_on && (!a.obj.mask || a.obj.mask[pi])) {
                const T pu[3] = {pv[1], pv[2], T(0)}, z3[3] = {0, 0, 0};
                jacc += obj_density<T>(a.obj, p[0], p[1], 0, (double)pv[0], pu, T(0), z3);
            }
        });
    }
    if (obj_on) store_partial(a.obj, jacc, blin, sh4);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd2d(const FwdArgs<T> a) {
    fwd2d_body<T>(a, blockIdx.x, blockIdx.y, blockIdx.x + (long long)blockIdx.y * gridDim.x);
}

// first tile of the job that owns flat tile b (tile0 ascending, tile0[0] = 0)
__device__ __forceinline__ int job_of(const long long *tile0, int njobs, long long b) {
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tile0[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// one launch for the current step of many jobs: flat tile b -> (job, local tile)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd2d_batch(const FwdArgs<T> *args, const long long *tile0,
                                                        int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of(tile0, njobs, b);
    const FwdArgs<T> &a = args[j];
    const long long t = b - tile0[j];
    const int nbx = (a.g.n[0] + TX - 1) / TX;
    fwd2d_body<T>(a, (int)(t % nbx), (int)(t / nbx), t);
}

// transposed difference operator along one axis at coordinate c: sum_r D[r][c] f(r), with f
// given for r = c-2 .. c+2 (rows off the grid are never read)
template <typename T>
__device__ __forceinline__ T deriv_T(const T f[5], int c, int n, int per) {
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

template <typename T>
__device__ __forceinline__ void adj2d_body(const AdjArgs<T> &a, int bx, int by) {
    constexpr int LX = TX + 8, LY = TY + 8;  // lambda, halo 4, origin (x0-4, y0-4)
    constexpr int PX = TX + 6, PY = TY + 6;  // P*, V*, halo 3, origin (x0-3, y0-3)
    constexpr int MX = TX + 4, MY = TY + 4;  // moments, halo 2, origin (x0-2, y0-2)
    constexpr int NBUF = (3 * LX * LY > 6 * MX * MY) ? 3 * LX * LY : 6 * MX * MY;
    __shared__ T sbuf[NBUF];  // lambda, then the moments
    __shared__ T sPV[3][PY][PX];

    const int tid = threadIdx.x;
    const int x0 = bx * TX, y0 = by * TY;
    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1];
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const bool kobj = obj_on && obj_uses_kappa(a.obj.kind);
    const double sc = a.obj.scale;
    T(*sl)[LY][LX] = reinterpret_cast<T(*)[LY][LX]>(sbuf);

    // lambda = Lambda^n + dj^n/dX^n on halo 4
    for (int i = tid; i < LX * LY; i += kBlock) {
        const int lx = i % LX, ly = i / LX;
        int gx = x0 - 4 + lx, gy = y0 - 4 + ly;
        T P = 0, Vx = 0, Vy = 0;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1])) {
            const long long idx = gx + gy * g.sy;
            P = a.Pin[idx];
            Vx = a.Vin[0][idx];
            Vy = a.Vin[1][idx];
            if (obj_on && (!a.obj.mask || a.obj.mask[idx])) {
                double kap = 0.0, us[3] = {0, 0, 0};
                if (kobj && in_box(a.m, 2, gx, gy, 0)) {
                    const long long bi = box_index(a.box, a.m, 2, gx, gy, 0);
                    kap = a.kbox[bi];
                    us[0] = a.usbox[0][bi];
                    us[1] = a.usbox[1][bi];
                }
                double dP, dV[3];
                obj_dstate(a.obj, gx, gy, 0, kap, us, dP, dV);
                P += (T)(sc * dP);
                Vx += (T)(sc * dV[0]);
                Vy += (T)(sc * dV[1]);
            }
        }
        sl[0][ly][lx] = P;
        sl[1][ly][lx] = Vx;
        sl[2][ly][lx] = Vy;
    }
    __syncthreads();

    // boundary transpose + force transpose on halo 3; kappa_bar on the tile's own nodes
    for (int i = tid; i < PX * PY; i += kBlock) {
        const int lx = i % PX, ly = i / PX;
        const int gxu = x0 - 3 + lx, gyu = y0 - 3 + ly;  // unwrapped
        int gx = gxu, gy = gyu;
        T P = 0, Vx = 0, Vy = 0;
        if (wrapc(gx, nx, g.per[0]) && wrapc(gy, ny, g.per[1]) && !on_face(g, 0, gx) &&
            !on_face(g, 1, gy)) {
            const int llx = lx + 1, lly = ly + 1;  // position in sl
            T acc[4] = {sl[0][lly][llx], sl[1][lly][llx], sl[2][lly][llx], T(0)};
            const int c[3] = {gx, gy, 0};
            gather_boundary_T<2>(g, a.bc.kind, c, acc, [&](const int p[3], int comp) -> T {
                return sl[comp][lly + (p[1] - gy)][llx + (p[0] - gx)];
            });
            const long long idx = gx + gy * g.sy;
            T kap = 0, us[3] = {0, 0, 0};
            const bool inb = in_box(a.m, 2, gx, gy, 0);
            long long bi = 0;
            if (inb) {
                bi = box_index(a.box, a.m, 2, gx, gy, 0);
                kap = a.kbox[bi];
                us[0] = a.usbox[0][bi];
                us[1] = a.usbox[1][bi];
            }
            const T ks = a.kstatic ? a.kstatic[idx] : T(0);
            const T inv = T(1) / (T(1) + kap + ks);
            P = acc[0];
            Vx = acc[1] * inv;
            Vy = acc[2] * inv;
            const bool own = lx >= 3 && lx < 3 + TX && ly >= 3 && ly < 3 + TY && gxu < nx && gyu < ny;
            if (own && inb) {
                const T ux = a.ucur[0][idx], uy = a.ucur[1][idx];
                double kb = -((double)Vx * ((double)ux - (double)us[0]) +
                              (double)Vy * ((double)uy - (double)us[1]));
                if (kobj && (!a.obj.mask || a.obj.mask[idx])) {
                    const double uu[3] = {(double)ux, (double)uy, 0.0};
                    const double uss[3] = {(double)us[0], (double)us[1], 0.0};
                    kb += sc * obj_dkappa(a.obj, gx, gy, 0, uu, uss);
                }
                a.kbar[bi] = (T)kb;
            }
        }
        sPV[0][ly][lx] = P;
        sPV[1][ly][lx] = Vx;
        sPV[2][ly][lx] = Vy;
    }
    __syncthreads();

    // pull transpose and the w-weighted moments (the paper's Eqs. arho, au, as) on halo 2
    T(*sm)[MY][MX] = reinterpret_cast<T(*)[MY][MX]>(sbuf);
    for (int i = tid; i < MX * MY; i += kBlock) {
        const int lx = i % MX, ly = i / MX;
        const int px = lx + 1, py = ly + 1;  // position in sPV
        T rt = 0, utx = 0, uty = 0, sxx = 0, sxy = 0, syy = 0;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int cx = d2q9::cx(q), cy = d2q9::cy(q);
            const T eb = sPV[0][py + cy][px + cx] + T(cx) * sPV[1][py + cy][px + cx] +
                         T(cy) * sPV[2][py + cy][px + cx];
            const T we = T(d2q9::wt(q)) * eb;
            rt += we;
            utx += T(cx) * we;
            uty += T(cy) * we;
            sxx += T(cx * cx) * we;
            sxy += T(cx * cy) * we;
            syy += T(cy * cy) * we;
        }
        sm[0][ly][lx] = rt;
        sm[1][ly][lx] = utx;
        sm[2][ly][lx] = uty;
        sm[3][ly][lx] = sxx;
        sm[4][ly][lx] = sxy;
        sm[5][ly][lx] = syy;
    }
    __syncthreads();

    // transposed equilibrium and strain: Lambda^{n-1}
    const T A2 = T(2) * a.A;
    for (int k = 0; k < (TX * TY) / kBlock; ++k) {
        const int lx = tid % TX, ly = tid / TX + k * (kBlock / TX);
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= nx || gy >= ny) continue;
        const long long idx = gx + gy * g.sy;
        const int mx = lx + 2, my = ly + 2;
        const T rt = sm[0][my][mx], utx = sm[1][my][mx], uty = sm[2][my][mx];
        const T sxx = sm[3][my][mx], sxy = sm[4][my][mx], syy = sm[5][my][mx];
        const T ux = a.uprev[0][idx], uy = a.uprev[1][idx];
        T vx = T(3) * utx + T(9) * (sxx * ux + sxy * uy) - T(3) * rt * ux;
        T vy = T(3) * uty + T(9) * (sxy * ux + syy * uy) - T(3) * rt * uy;
        // V_a += 2A sum_b D_b^T s~_ab
        T f[5];
#pragma unroll
        for (int o = 0; o < 5; ++o) f[o] = sm[3][my][mx + o - 2];
        vx += A2 * deriv_T(f, gx, nx, g.per[0]);
#pragma unroll
        for (int o = 0; o < 5; ++o) f[o] = sm[4][my + o - 2][mx];
        vx += A2 * deriv_T(f, gy, ny, g.per[1]);
#pragma unroll
        for (int o = 0; o < 5; ++o) f[o] = sm[4][my][mx + o - 2];
        vy += A2 * deriv_T(f, gx, nx, g.per[0]);
#pragma unroll
        for (int o = 0; o < 5; ++o) f[o] = sm[5][my + o - 2][mx];
        vy += A2 * deriv_T(f, gy, ny, g.per[1]);
        a.Pout[idx] = rt;
        a.Vout[0][idx] = vx;
        a.Vout[1][idx] = vy;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj2d(const AdjArgs<T> a) {
    adj2d_body<T>(a, blockIdx.x, blockIdx.y);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj2d_batch(const AdjArgs<T> *args, const long long *tile0,
                                                        int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of(tile0, njobs, b);
    const AdjArgs<T> &a = args[j];
    const long long t = b - tile0[j];
    const int nbx = (a.g.n[0] + TX - 1) / TX;
    adj2d_body<T>(a, (int)(t % nbx), (int)(t / nbx));
}

template <typename T>
hipError_t launch_fwd2d(const FwdArgs<T> &a, hipStream_t s) {
    dim3 grid((a.g.n[0] + TX - 1) / TX, (a.g.n[1] + TY - 1) / TY);
    hipLaunchKernelGGL(k_fwd2d<T>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adj2d(const AdjArgs<T> &a, hipStream_t s) {
    dim3 grid((a.g.n[0] + TX - 1) / TX, (a.g.n[1] + TY - 1) / TY);
    hipLaunchKernelGGL(k_adj2d<T>, grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

long long fwd_blocks(const Geom &g, int lattice, int esz) {
    if (g.dim == 2) return (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY);
    return fwd_blocks3d(g, lattice, esz);
}

long long tiles2d(const Geom &g) { return (long long)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY); }

template <typename T>
hipError_t launch_fwd2d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fwd2d_batch<T>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, args, tile0, njobs);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_adj2d_batch(const AdjArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, hipStream_t s) {
    if (njobs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj2d_batch<T>, dim3((unsigned)ntiles), dim3(kBlock), 0, s, args, tile0, njobs);
    return hipGetLastError();
}
template hipError_t launch_fwd2d_batch<float>(const FwdArgs<float> *, const long long *, int, long long, hipStream_t);
template hipError_t launch_fwd2d_batch<double>(const FwdArgs<double> *, const long long *, int, long long, hipStream_t);
template hipError_t launch_adj2d_batch<float>(const AdjArgs<float> *, const long long *, int, long long, hipStream_t);
template hipError_t launch_adj2d_batch<double>(const AdjArgs<double> *, const long long *, int, long long, hipStream_t);

template hipError_t launch_fwd2d<float>(const FwdArgs<float> &, hipStream_t);
template hipError_t launch_fwd2d<double>(const FwdArgs<double> &, hipStream_t);
template hipError_t launch_adj2d<float>(const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adj2d<double>(const AdjArgs<double> &, hipStream_t);

}  // namespace lks

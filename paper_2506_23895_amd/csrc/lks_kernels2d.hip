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

// Forward step as wave strips marching along y.  Lane l of wave w holds column
// c = 60 * strip - 2 + l; lanes 2..61 produce outputs, lanes 0, 1, 62, 63 are the column halo.
// A wave owns RY output rows: it issues the loads of every velocity row it needs (RY + 5) and
// every density row (RY + 2) into registers up front, then walks the rows as they arrive.  Per
// row r the lane evaluates the strain and the nine E_i of its own node once, adds the ones pulled
// by its own column (c_x = 0) into three in-flight output rows, and sums per target row the ones
// pulled by column c+1 (c_x = +1) and by column c-1 (c_x = -1); those sums reach the neighbouring
// lanes through one lane shift each when their target row completes.
#ifndef LKS_FWD2D_RY
#define LKS_FWD2D_RY 4
#endif
constexpr int SW = 60;            // output columns per wave strip
constexpr int RY = LKS_FWD2D_RY;  // output rows per wave
constexpr int WPB = kBlock / 64;

// face nodes written from interior node (c, o), with their objective contribution
template <typename T>
__device__ __noinline__ double fwd2d_push(const FwdArgs<T> &a, int c, int o, T rs, T nux, T nuy,
                                          bool obj_on) {
    const Geom &g = a.g;
    double j = 0.0;
    const int c3[3] = {c, o, 0};
    const T v[4] = {rs, nux, nuy, T(0)};
    push_boundary<T, 2>(g, a.bc, c3, v, [&](const int p[3], const T pv[4]) {
        const long long pi = p[0] + p[1] * g.sy;
        a.rout[pi] = pv[0];
        a.uout[0][pi] = pv[1];
        a.uout[1][pi] = pv[2];
        if (obj_on && !obj_uses_kappa(a.obj.kind) && (!a.obj.mask || a.obj.mask[pi])) {
            const T pu[3] = {pv[1], pv[2], T(0)}, z3[3] = {0, 0, 0};
            j += obj_density<T>(a.obj, p[0], p[1], 0, (double)pv[0], pu, T(0), z3);
        }
    });
    return j;
}

template <typename T>
__device__ __forceinline__ void fwd2d_body(const FwdArgs<T> &a, int bx, int by, long long slot0) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1];
    const int strip = bx * WPB + w;
    const long long pslot = slot0 + w;
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const int nstrips = (nx + SW - 1) / SW;
    if (strip >= nstrips) {
        if (obj_on && lane == 0) a.obj.partials[pslot] = 0.0;
        return;
    }
    const int c = strip * SW - 2 + lane;
    int cw = c;
    const bool cin = wrapc(cw, nx, g.per[0]);
    const int cmin = strip * SW - 2, cmax = cmin + 63;
    const bool xface = !g.per[0] && ((cmin <= 0 && 0 <= cmax) || (cmin <= nx - 1 && nx - 1 <= cmax));
    const bool out_lane = lane >= 2 && lane < 62 && c < nx && !on_face(g, 0, c);
    const int y0 = by * RY;
    const T *__restrict__ ux_in = a.uin[0];
    const T *__restrict__ uy_in = a.uin[1];
    const T *__restrict__ r_in = a.rin;
    // does this wave's rectangle meet the footprint box (wave-uniform)?
    const bool wbox = a.m.hi[0] >= strip * SW && a.m.lo[0] < strip * SW + SW && a.m.hi[1] >= y0 &&
                      a.m.lo[1] < y0 + RY;

    // every row this wave needs, requested before any arithmetic
    T ux[RY + 5], uy[RY + 5], rv[RY + 2];
    T kb[RY], sbx[RY], sby[RY];  // kappa, u_S of the output rows (footprint waves only)
#pragma unroll
    for (int k = 0; k < RY; ++k) {
        kb[k] = sbx[k] = sby[k] = T(0);
        const int o = y0 + k;
        if (wbox && c >= a.m.lo[0] && c <= a.m.hi[0] && o >= a.m.lo[1] && o <= a.m.hi[1]) {
            const long long bi = box_index(a.box, a.m, 2, c, o, 0);
            kb[k] = a.kin[bi];
            sbx[k] = a.usin[0][bi];
            sby[k] = a.usin[1][bi];
        }
    }
#pragma unroll
    for (int k = 0; k < RY + 5; ++k) {
        int yw = y0 - 3 + k;
        ux[k] = uy[k] = T(0);
        if (cin && wrapc(yw, ny, g.per[1])) {
            const long long idx = cw + yw * g.sy;
            ux[k] = ux_in[idx];
            uy[k] = uy_in[idx];
        }
    }
#pragma unroll
    for (int k = 0; k < RY + 2; ++k) {
        int yw = y0 - 1 + k;
        rv[k] = T(0);
        if (cin && wrapc(yw, ny, g.per[1])) rv[k] = r_in[cw + yw * g.sy];
    }

    T acc_r[3] = {0, 0, 0}, acc_m[3] = {0, 0, 0};  // own column: rho*, m_y* for rows r-1, r, r+1
    T trr[3] = {0, 0, 0}, trm[3] = {0, 0, 0};      // pulled by column c+1
    T tlr[3] = {0, 0, 0}, tlm[3] = {0, 0, 0};      // pulled by column c-1
    double jacc = 0.0;
    const T A2 = T(2) * a.A;
    const T wa = T(d2q9::WA), wd = T(d2q9::WD), w0 = T(d2q9::W0);

#pragma unroll
    for (int e = 0; e < RY + 2; ++e) {
        const int r = y0 - 1 + e;  // row of the E_i evaluated now; u rows r-2..r+2 = ux[e..e+4]
        int rw = r;
        if (wrapc(rw, ny, g.per[1])) {  // wave-uniform
            const T uxc = ux[e + 2], uyc = uy[e + 2];
            const T uxl = from_left(uxc), uxr = from_right(uxc);
            const T uyl = from_left(uyc), uyr = from_right(uyc);
            T dxux = T(0.5) * (uxr - uxl), dxuy = T(0.5) * (uyr - uyl);
            if (xface) {
                const T uxll = from_left(uxl), uxrr = from_right(uxr);
                const T uyll = from_left(uyl), uyrr = from_right(uyr);
                if (c == 0) {
                    dxux = T(-1.5) * uxc + T(2) * uxr - T(0.5) * uxrr;
                    dxuy = T(-1.5) * uyc + T(2) * uyr - T(0.5) * uyrr;
                } else if (c == nx - 1) {
                    dxux = T(1.5) * uxc - T(2) * uxl + T(0.5) * uxll;
                    dxuy = T(1.5) * uyc - T(2) * uyl + T(0.5) * uyll;
                }
            }
            T dyux, dyuy;
            if (!g.per[1] && rw == 0) {
                dyux = T(-1.5) * uxc + T(2) * ux[e + 3] - T(0.5) * ux[e + 4];
                dyuy = T(-1.5) * uyc + T(2) * uy[e + 3] - T(0.5) * uy[e + 4];
            } else if (!g.per[1] && rw == ny - 1) {
                dyux = T(1.5) * uxc - T(2) * ux[e + 1] + T(0.5) * ux[e];
                dyuy = T(1.5) * uyc - T(2) * uy[e + 1] + T(0.5) * uy[e];
            } else {
                dyux = T(0.5) * (ux[e + 3] - ux[e + 1]);
                dyuy = T(0.5) * (uy[e + 3] - uy[e + 1]);
            }
            const T a0 = rv[e] - T(1.5) * (uxc * uxc + uyc * uyc);
            const T bx3 = T(3) * uxc, by3 = T(3) * uyc;
            const T txx = T(4.5) * uxc * uxc + A2 * dxux;
            const T tyy = T(4.5) * uyc * uyc + A2 * dyuy;
            const T txy2 = T(9) * uxc * uyc + A2 * (dyux + dxuy);
            const T q = a0 + txx + tyy;
            const T m = cin ? T(1) : T(0);  // nothing from columns outside the domain
            const T e0 = m * w0 * a0;
            const T e1 = m * wa * (a0 + bx3 + txx), e3 = m * wa * (a0 - bx3 + txx);
            const T e2 = m * wa * (a0 + by3 + tyy), e4 = m * wa * (a0 - by3 + tyy);
            const T e5 = m * wd * (q + bx3 + by3 + txy2), e6 = m * wd * (q - bx3 + by3 - txy2);
            const T e7 = m * wd * (q - bx3 - by3 + txy2), e8 = m * wd * (q + bx3 - by3 - txy2);
            acc_r[1] += e0;
            acc_r[2] += e2;
            acc_m[2] += e2;
            acc_r[0] += e4;
            acc_m[0] -= e4;
            trr[1] += e1;
            trr[2] += e5;
            trm[2] += e5;
            trr[0] += e8;
            trm[0] -= e8;
            tlr[1] += e3;
            tlr[2] += e6;
            tlm[2] += e6;
            tlr[0] += e7;
            tlm[0] -= e7;
        }
        if (e >= 2) {  // output row o = r - 1 (rows y0 .. y0 + RY - 1) is complete
            const int o = r - 1;
            const T fr = from_left(trr[0]), fm = from_left(trm[0]);
            const T gr = from_right(tlr[0]), gm = from_right(tlm[0]);
            if (out_lane && o < ny && !on_face(g, 1, o)) {
                const T rs = acc_r[0] + fr + gr, mx = fr - gr, my = acc_m[0] + fm + gm;
                const T kap = kb[e - 2];
                const T us0 = sbx[e - 2], us1 = sby[e - 2];
                const long long idx = c + o * g.sy;
                const T ks = a.kstatic ? a.kstatic[idx] : T(0);
                const T inv = T(1) / (T(1) + kap + ks);
                const T nux = (mx + kap * us0 + a.gf[0]) * inv;
                const T nuy = (my + kap * us1 + a.gf[1]) * inv;
                a.rout[idx] = rs;
                a.uout[0][idx] = nux;
                a.uout[1][idx] = nuy;
                if (obj_on && (kap != T(0) || !obj_uses_kappa(a.obj.kind)) && (!a.obj.mask || a.obj.mask[idx])) {
                    const T uv[3] = {nux, nuy, T(0)}, usv[3] = {us0, us1, T(0)};
                    jacc += obj_density<T>(a.obj, c, o, 0, (double)rs, uv, kap, usv);
                }
                if (c == 1 || c == nx - 2 || o == 1 || o == ny - 2)
                    jacc += fwd2d_push<T>(a, c, o, rs, nux, nuy, obj_on);
            }
        }
        acc_r[0] = acc_r[1]; acc_r[1] = acc_r[2]; acc_r[2] = T(0);
        acc_m[0] = acc_m[1]; acc_m[1] = acc_m[2]; acc_m[2] = T(0);
        trr[0] = trr[1]; trr[1] = trr[2]; trr[2] = T(0);
        trm[0] = trm[1]; trm[1] = trm[2]; trm[2] = T(0);
        tlr[0] = tlr[1]; tlr[1] = tlr[2]; tlr[2] = T(0);
        tlm[0] = tlm[1]; tlm[1] = tlm[2]; tlm[2] = T(0);
    }
    if (obj_on) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) jacc += __shfl_xor(jacc, o, 64);
        if (lane == 0) a.obj.partials[pslot] = jacc;
    }
}

__host__ __device__ inline int fwd2d_grid_x(const Geom &g) {
    const int nstrips = (g.n[0] + SW - 1) / SW;
    return (nstrips + WPB - 1) / WPB;
}
__host__ __device__ inline int fwd2d_grid_y(const Geom &g) { return (g.n[1] + RY - 1) / RY; }

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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd2d_batch(const FwdArgs<T> *args, const long long *tile0,
                                                        int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of(tile0, njobs, b);
    const FwdArgs<T> &a = args[j];
    const long long t = b - tile0[j];
    const long long ns = (a.mode & FWD_STENCIL) ? (long long)fwd2d_grid_x(a.g) * fwd2d_grid_y(a.g) : 0;
    if (t >= ns) {  // extra blocks: transfer of the next step onto its footprint box
        transfer_box<T, 2, kBlock>(a.des, a.mnext, a.box, a.knext, a.usnext, t - ns);
        return;
    }
    const int nbx = fwd2d_grid_x(a.g);
    fwd2d_body<T>(a, (int)(t % nbx), (int)(t / nbx), t * WPB);
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
__global__ __launch_bounds__(kBlock) void k_adj2d_batch(const AdjArgs<T> *args, const long long *tile0,
                                                        int njobs) {
    const long long b = blockIdx.x;
    const int j = job_of(tile0, njobs, b);
    const AdjArgs<T> &a = args[j];
    const long long t = b - tile0[j];
    const int nbx = (a.g.n[0] + TX - 1) / TX;
    adj2d_body<T>(a, (int)(t % nbx), (int)(t / nbx));
}

long long fwd_blocks(const Geom &g, int lattice, int esz) {
    // one objective partial per wave (2D) or per block (3D)
    if (g.dim == 2) return (long long)fwd2d_grid_x(g) * fwd2d_grid_y(g) * WPB;
    return fwd_blocks3d(g, lattice, esz);
}

long long xfer_blocks(int dim, long long cells, int esz) {
    if (dim == 2) return (cells + kBlock - 1) / kBlock;
    return xfer_blocks3d(cells, esz);
}

long long tiles2d_fwd(const Geom &g) { return (long long)fwd2d_grid_x(g) * fwd2d_grid_y(g); }
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


}  // namespace lks

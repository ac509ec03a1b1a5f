// 2D D2Q9 kernels: one fused forward step and one fused adjoint step per launch, both on wave
// strips: the 64 lanes of a wave hold 64 consecutive columns and the wave walks a few rows, so
// x-neighbours are one lane away (DPP row shifts) and y-neighbours are registers of the same lane.
// Each launch is a list of work units, one per wave, sized so that no kind of wave outlives the
// rest: interior units (no face, no wrap) run compiled-out variants, units of a strip that holds
// an x face run the XF variants (that one face's rule inline), and the rows next to the y faces
// (or a periodic axis's wrap) run the general variants with the composite boundary rules.
//
// Forward step (Algorithm 1 body, Sec. 2.2-2.3): lanes 2..61 own output columns, the two lanes on
// each side are the u halo.  Every row the wave needs (u with halo 2, rho - 1 with halo 1, kappa
// and u_S of its output rows from the footprint store) is requested before any arithmetic; then,
// row by row, the strain (central differences, one-sided on non-periodic faces) and the
// equilibrium E_i, whose pulled parts land in three in-flight output rows; the VPM update, the
// composite boundary rules of the face nodes that copy from this node, and one FP64 objective
// partial per wave.  Extra blocks of the same launch transfer the next step onto its footprint box.
// Adjoint step (the exact transpose, in reverse order): lanes 3..60 own output columns.  Per row,
// lambda = Lambda + dj/dX, the boundary and force transposes give (P*, V*) and kappa_bar on the
// footprint box; the w-weighted moments (rho~, u~, s~) of the pull transpose
// E~_i(y) = P*(y+c_i) + c_i.V*(y+c_i) factor into an x-stencil (lane shifts) and a y-stencil
// (registers); then Lambda^{n-1} from the transposed equilibrium and strain operator.  Extra blocks
// of the same launch run the sensitivity gather of the step after it.
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

// Forward step as wave strips marching along y.  Lane l of wave w holds column
// c = 60 * strip - 2 + l; lanes 2..61 produce outputs, lanes 0, 1, 62, 63 are the column halo.
// A wave owns NR output rows (RY in the interior, RF next to faces): it issues the loads of every
// velocity row it needs (NR + 5) and every density row (NR + 2) into registers up front, then
// walks the rows as they arrive.  Per
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
        gst(a.rout)[pi] = pv[0];
        gst(a.uout[0])[pi] = pv[1];
        gst(a.uout[1])[pi] = pv[2];
        if (obj_on && !obj_uses_kappa(a.obj.kind) && (!a.obj.mask || a.obj.mask[pi])) {
            const T pu[3] = {pv[1], pv[2], T(0)}, z3[3] = {0, 0, 0};
            j += obj_density<T>(a.obj, p[0], p[1], 0, (double)pv[0], pu, T(0), z3);
        }
    });
    return j;
}

__device__ __forceinline__ float rcp_t(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp_t(double v) { return 1.0 / v; }

// IN: the wave touches no face, needs no periodic wrap and every E row it evaluates has central
// differences on both axes (decided per wave), so the bounds, wrap, one-sided and boundary-push
// code is compiled out.
template <typename T, bool IN, int NR, bool XF = false>
__device__ __forceinline__ void fwd2d_rows(const FwdArgs<T> &a, int strip, int y0, long long pslot,
                                           bool obj_on) {
    const int lane = threadIdx.x & 63;
    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1];
    const int c = strip * SW - 2 + lane;
    // XF (with IN): a strip that holds an x face, x not periodic, rows as IN.  Loads come from the
    // clamped column, columns off the grid contribute nothing, the face columns take one-sided
    // x-derivatives, and the lane next to a face writes the face node by that face's rule.
    const int cl = XF ? min(max(c, 0), nx - 1) : c;
    const bool cval = !XF || cl == c;
    int cw = c;
    const bool cin = IN ? cval : wrapc(cw, nx, g.per[0]);
    const int cmin = strip * SW - 2, cmax = cmin + 63;
    const bool xface = !IN && !g.per[0] && ((cmin <= 0 && 0 <= cmax) || (cmin <= nx - 1 && nx - 1 <= cmax));
    const bool out_lane = lane >= 2 && lane < 62 &&
                          (IN ? (!XF || (cval && c != 0 && c != nx - 1)) : (c < nx && !on_face(g, 0, c)));
    const LKS_GLOBAL T *__restrict__ ux_in = gld(a.uin[0]);
    const LKS_GLOBAL T *__restrict__ uy_in = gld(a.uin[1]);
    const LKS_GLOBAL T *__restrict__ r_in = gld(a.rin);
    LKS_GLOBAL T *__restrict__ r_out = gst(a.rout);
    LKS_GLOBAL T *__restrict__ ux_out = gst(a.uout[0]);
    LKS_GLOBAL T *__restrict__ uy_out = gst(a.uout[1]);
    const LKS_GLOBAL T *__restrict__ kst = gld(a.kstatic);
    const LKS_GLOBAL uint8_t *__restrict__ omask = gld(a.obj.mask);
    // does this wave's rectangle meet the footprint box (wave-uniform)?
    const bool wbox = a.m.hi[0] >= strip * SW && a.m.lo[0] < strip * SW + SW && a.m.hi[1] >= y0 &&
                      a.m.lo[1] < y0 + NR;
    const bool brink = wbox || a.kstatic != nullptr;  // kappa + kappa_s can be non-zero here

    // every row this wave needs, requested before any arithmetic
    T ux[NR + 5], uy[NR + 5], rv[NR + 2];
    T kb[NR], sbx[NR], sby[NR];  // kappa, u_S of the output rows (footprint waves only)
#pragma unroll
    for (int k = 0; k < NR + 5; ++k) {
        int yw = y0 - 3 + k;
        ux[k] = uy[k] = T(0);
        if (IN) {
            if (k == 0) continue;  // the one-sided stencils that read row y0 - 3 never run here
            const long long idx = cl + (long long)yw * g.sy;
            const T v0 = ux_in[idx], v1 = uy_in[idx];
            ux[k] = cval ? v0 : T(0);
            uy[k] = cval ? v1 : T(0);
        } else {
            const bool ok = cin && wrapc(yw, ny, g.per[1]);
            const long long idx = ok ? cw + (long long)yw * g.sy : 0;
            const T v0 = ux_in[idx], v1 = uy_in[idx];
            ux[k] = ok ? v0 : T(0);
            uy[k] = ok ? v1 : T(0);
        }
    }
#pragma unroll
    for (int k = 0; k < NR + 2; ++k) {
        int yw = y0 - 1 + k;
        rv[k] = T(0);
        if (IN) {
            const T v = r_in[cl + (long long)yw * g.sy];
            rv[k] = cval ? v : T(0);
        } else {
            const bool ok = cin && wrapc(yw, ny, g.per[1]);
            const T v = r_in[ok ? cw + (long long)yw * g.sy : 0];
            rv[k] = ok ? v : T(0);
        }
    }

    // kappa, u_S last, in one block: every index comes from clamped coordinates (no per-lane
    // branch), all loads are issued before the first select, and the field rows above are already
    // in flight while they wait
#pragma unroll
    for (int k = 0; k < NR; ++k) kb[k] = sbx[k] = sby[k] = T(0);
    if (wbox) {  // wave-uniform
        T k0[NR], s0[NR], s1[NR];
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const int bi = box_index2_clamped(a.box, a.m, c, y0 + k);
            k0[k] = gld(a.kin)[bi];
            s0[k] = gld(a.usin[0])[bi];
            s1[k] = gld(a.usin[1])[bi];
        }
#pragma unroll
        for (int k = 0; k < NR; ++k) {
            const bool inb = in_box(a.m, 2, c, y0 + k, 0);
            kb[k] = inb ? k0[k] : T(0);
            sbx[k] = inb ? s0[k] : T(0);
            sby[k] = inb ? s1[k] : T(0);
        }
    }

    T acc_r[3] = {0, 0, 0}, acc_m[3] = {0, 0, 0};  // own column: rho*, m_y* for rows r-1, r, r+1
    T trr[3] = {0, 0, 0}, trm[3] = {0, 0, 0};      // pulled by column c+1
    T tlr[3] = {0, 0, 0}, tlm[3] = {0, 0, 0};      // pulled by column c-1
    double jacc = 0.0;
    const T A = a.A;
    const T wa = T(d2q9::WA), wd = T(d2q9::WD), w0 = T(d2q9::W0);

#pragma unroll
    for (int e = 0; e < NR + 2; ++e) {
        const int r = y0 - 1 + e;  // row of the E_i evaluated now; u rows r-2..r+2 = ux[e..e+4]
        int rw = r;
        if (IN || wrapc(rw, ny, g.per[1])) {  // wave-uniform
            const T uxc = ux[e + 2], uyc = uy[e + 2];
            const T uxl = from_left(uxc), uxr = from_right(uxc);
            const T uyl = from_left(uyc), uyr = from_right(uyc);
            // twice the derivatives: central (f+ - f-), one-sided 2 (-1.5 f0 + 2 f1 - 0.5 f2)
            T gxux = uxr - uxl, gxuy = uyr - uyl;
            if ((!IN && xface) || XF) {
                const T uxll = from_left(uxl), uxrr = from_right(uxr);
                const T uyll = from_left(uyl), uyrr = from_right(uyr);
                if (c == 0) {
                    gxux = T(-3) * uxc + T(4) * uxr - uxrr;
                    gxuy = T(-3) * uyc + T(4) * uyr - uyrr;
                } else if (c == nx - 1) {
                    gxux = T(3) * uxc - T(4) * uxl + uxll;
                    gxuy = T(3) * uyc - T(4) * uyl + uyll;
                }
            }
            T gyux = ux[e + 3] - ux[e + 1], gyuy = uy[e + 3] - uy[e + 1];
            if (!IN && !g.per[1] && rw == 0) {
                gyux = T(-3) * uxc + T(4) * ux[e + 3] - ux[e + 4];
                gyuy = T(-3) * uyc + T(4) * uy[e + 3] - uy[e + 4];
            } else if (!IN && !g.per[1] && rw == ny - 1) {
                gyux = T(3) * uxc - T(4) * ux[e + 1] + ux[e];
                gyuy = T(3) * uyc - T(4) * uy[e + 1] + uy[e];
            }
            const T a0 = rv[e] - T(1.5) * (uxc * uxc + uyc * uyc);
            const T bx3 = T(3) * uxc, by3 = T(3) * uyc;
            const T txx = T(4.5) * uxc * uxc + A * gxux;
            const T tyy = T(4.5) * uyc * uyc + A * gyuy;
            const T txy2 = T(9) * uxc * uyc + A * (gyux + gxuy);
            const T q = a0 + txx + tyy;
            const T m = cin ? T(1) : T(0);  // nothing from columns outside the domain
            T e0 = w0 * a0;
            T e1 = wa * (a0 + bx3 + txx), e3 = wa * (a0 - bx3 + txx);
            T e2 = wa * (a0 + by3 + tyy), e4 = wa * (a0 - by3 + tyy);
            T e5 = wd * (q + bx3 + by3 + txy2), e6 = wd * (q - bx3 + by3 - txy2);
            T e7 = wd * (q - bx3 - by3 + txy2), e8 = wd * (q + bx3 - by3 - txy2);
            if (!IN || XF) {
                e0 *= m; e1 *= m; e2 *= m; e3 *= m; e4 *= m;
                e5 *= m; e6 *= m; e7 *= m; e8 *= m;
            }
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
        if (e >= 2) {  // output row o = r - 1 (rows y0 .. y0 + NR - 1) is complete
            const int o = r - 1;
            const T fr = from_left(trr[0]), fm = from_left(trm[0]);
            const T gr = from_right(tlr[0]), gm = from_right(tlm[0]);
            if (out_lane && (IN || (o < ny && !on_face(g, 1, o)))) {
                const T rs = acc_r[0] + fr + gr, mx = fr - gr, my = acc_m[0] + fm + gm;
                const T kap = kb[e - 2];
                const T us0 = sbx[e - 2], us1 = sby[e - 2];
                const long long idx = c + (long long)o * g.sy;
                T nux = mx + a.gf[0], nuy = my + a.gf[1];
                if (brink) {
                    const T ks = kst ? kst[idx] : T(0);
                    const T inv = rcp_t(T(1) + kap + ks);
                    nux = (nux + kap * us0) * inv;
                    nuy = (nuy + kap * us1) * inv;
                }
                r_out[idx] = rs;
                ux_out[idx] = nux;
                uy_out[idx] = nuy;
                if (obj_on && (kap != T(0) || !obj_uses_kappa(a.obj.kind)) && (!omask || omask[idx])) {
                    const T uv[3] = {nux, nuy, T(0)}, usv[3] = {us0, us1, T(0)};
                    jacc += obj_density<T>(a.obj, c, o, 0, (double)rs, uv, kap, usv);
                }
                if (!IN && (c == 1 || c == nx - 2 || o == 1 || o == ny - 2))
                    jacc += fwd2d_push<T>(a, c, o, rs, nux, nuy, obj_on);
                if (XF && (c == 1 || c == nx - 2)) {  // the face node next to this one
                    const int f = c == 1 ? 0 : 1, kind = a.bc.kind[f], pc = c == 1 ? 0 : nx - 1;
                    const T pr = bc_copies(kind, 0, 0) ? rs : a.bc.rho[f];
                    const T pux = bc_copies(kind, 1, 0) ? nux : a.bc.u[f][0];
                    const T puy = bc_copies(kind, 2, 0) ? nuy : a.bc.u[f][1];
                    const long long pi = pc + (long long)o * g.sy;
                    r_out[pi] = pr;
                    ux_out[pi] = pux;
                    uy_out[pi] = puy;
                    if (obj_on && !obj_uses_kappa(a.obj.kind) && (!omask || omask[pi])) {
                        const T pu[3] = {pux, puy, T(0)}, z3[3] = {T(0), T(0), T(0)};
                        jacc += obj_density<T>(a.obj, pc, o, 0, (double)pr, pu, T(0), z3);
                    }
                }
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
        // objectives weighted by kappa vanish off the footprint: a wave that does not meet it
        // stores its exact sum, +0, without the cross-lane reduction
        if (!wbox && obj_uses_kappa(a.obj.kind)) {
            if (lane == 0) gst(a.obj.partials)[pslot] = 0.0;
        } else {
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) jacc += __shfl_xor(jacc, o, 64);
            if (lane == 0) gst(a.obj.partials)[pslot] = jacc;
        }
    }
}

// Work units of one 2D forward step, one per wave, in row bands.  Over rows [2, yhi), in chunks of
// RY rows, every strip is one unit: inner strips (lanes 0..63 inside the grid, no wrap) with the
// compiled-out interior variant, outer strips that hold an x face (x not periodic) with the XF
// variant.  Every other (strip, row pair) — the rows next to the y faces (or a periodic y's wrap),
// and all rows of the outer strips when x is periodic — is a unit of RF rows with the general
// variant (wraps, one-sided derivatives, composite boundary pushes), half the height so that those
// waves take about as long as the others.  Unit order: the rows [0, 2) of every strip, then per
// chunk its units (inner strips, then outer ones), then the rows [yhi, ny).  Without inner strips
// or chunks every unit is general.  Unit k owns objective partial slot k.
constexpr int RF = 2;
static_assert(RY >= RF && RY % RF == 0, "an outer strip's chunk of RY rows is RY / RF general units of RF rows");
struct Fwd2dUnits {
    int nstrips, ninner, nmc, yhi, ngs, nxf, band;
    long long top, mid, total;
};
__host__ __device__ inline Fwd2dUnits fwd2d_units(const Geom &g) {
    Fwd2dUnits u;
    const int nx = g.n[0], ny = g.n[1];
    u.nstrips = (nx + SW - 1) / SW;
    u.nmc = ny >= 4 + RY ? (ny - 4) / RY : 0;
    u.ninner = (u.nmc > 0 && nx >= 2 * SW + 2) ? (nx - 62) / SW : 0;
    if (u.ninner == 0) u.nmc = 0;
    u.ngs = u.nstrips - u.ninner;
    u.nxf = g.per[0] ? 0 : u.ngs;  // outer strips with an XF unit per chunk
    u.band = u.ninner + (u.nxf > 0 ? u.nxf : (RY / RF) * u.ngs);
    u.yhi = u.nmc > 0 ? 2 + RY * u.nmc : 0;
    u.top = u.nmc > 0 ? (long long)u.nstrips : 0;
    u.mid = (long long)u.nmc * u.band;
    u.total = u.top + u.mid + (long long)u.nstrips * ((ny - u.yhi + RF - 1) / RF);
    return u;
}
__host__ __device__ inline long long fwd2d_nblocks(const Geom &g) { return (fwd2d_units(g).total + WPB - 1) / WPB; }

template <typename T>
__device__ __forceinline__ void fwd2d_unit(const FwdArgs<T> &a, const Fwd2dUnits &u, long long k) {
    const int lane = threadIdx.x & 63;
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    if (k >= u.total) {  // padding wave of the last block
        if (obj_on && lane == 0) gst(a.obj.partials)[k] = 0.0;
        return;
    }
    int strip, y0;
    if (k >= u.top && k < u.top + u.mid) {
        const int kk = (int)(k - u.top);
        const int c = kk / u.band, m = kk % u.band;
        if (m < u.ninner) {
            fwd2d_rows<T, true, RY>(a, 1 + m, 2 + RY * c, k, obj_on);
            return;
        }
        const int gq = m - u.ninner;
        if (u.nxf > 0) {
            fwd2d_rows<T, true, RY, true>(a, gq == 0 ? 0 : u.ninner + gq, 2 + RY * c, k, obj_on);
            return;
        }
        const int q = gq % u.ngs;
        strip = q == 0 ? 0 : u.ninner + q;
        y0 = 2 + RY * c + RF * (gq / u.ngs);
    } else {
        const int kk = (int)(k < u.top ? k : k - u.top - u.mid);
        strip = kk % u.nstrips;
        y0 = (k < u.top ? 0 : u.yhi) + RF * (kk / u.nstrips);
    }
    fwd2d_rows<T, false, RF>(a, strip, y0, k, obj_on);
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

template <typename T>
__global__ __launch_bounds__(kBlock) void k_fwd2d_batch(const FwdArgs<T> *__restrict__ args, const long long *__restrict__ tile0,
                                                        int njobs) {
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of(tile0, njobs, b));
    const FwdArgs<T> &a = args[j];
    touch_lines<sizeof(FwdArgs<T>)>(&a);
    const long long t = njobs == 1 ? b : b - tile0[j];  // one job: tile0 = {0}
    const Fwd2dUnits u = fwd2d_units(a.g);
    const long long ns = (a.mode & FWD_STENCIL) ? (u.total + WPB - 1) / WPB : 0;
    // Extra blocks transfer the next step onto its footprint box.  LIN blocks are short and come
    // after the stencil tiles, in its tail; the cosine kernel's blocks are long enough to set the
    // tail there, so they come first and overlap the stencil waves (1024^2 forward: COS4 16.0 ->
    // 13.4 us; LIN first would cost 11.7 -> 12.3 us).  The order is a bit of the mode word, which
    // the tiles read anyway: a further argument load would lengthen every tile's start.
    long long ts = t;
    if (a.mode & FWD_TRANSFER_FIRST) {
        const long long nx = (a.mode & FWD_TRANSFER_NEXT) ? (a.box.cells + kBlock - 1) / kBlock : 0;
        if (t < nx) {
            transfer_box<T, 2, kBlock>(a.des, a.mnext, a.box, a.knext, a.usnext, t);
            return;
        }
        ts = t - nx;
    } else if (t >= ns) {
        transfer_box<T, 2, kBlock>(a.des, a.mnext, a.box, a.knext, a.usnext, t - ns);
        return;
    }
    // XCD-aware: each XCD takes a contiguous run of blocks (neighbouring row bands share halos)
    const long long tl = xcd_tile(ts, ns);
    fwd2d_unit<T>(a, u, tl * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    prefetch_next<sizeof(FwdArgs<T>)>(a.next);
}

// transposed difference operator along one axis at coordinate c: sum_r D[r][c] f(r), with f
// given for r = c-2 .. c+2 (rows off the grid are never read)
template <typename T>
__device__ __forceinline__ T deriv_T(const T f[5], int c, int n, int per) {
    // rows c-2 .. c+2 all use central differences: only D[c-1][c] = 1/2 and D[c+1][c] = -1/2
    if (per || (c >= 3 && c <= n - 4)) return T(0.5) * (f[1] - f[3]);
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

// Adjoint step as wave strips marching along y, the transpose of the forward step taken in
// reverse order.  Lane l of a wave holds column c = 58 * strip - 3 + l; lanes 3..60 produce
// outputs.  Per row of the wave's window:
//   lambda = Lambda^n + dj^n/dX^n                        (loaded rows, objective added)
//   (P*, V*) = boundary transpose of lambda, V* / (1 + kappa + kappa_s), zero on face nodes;
//   kappa_bar = -V*.(u^n - u_S) + dj/dkappa on the wave's own footprint nodes
//   moments of E~_i(y) = P*(y + c_i) + c_i.V*(y + c_i) with weights w_i c_i^a c_i^b: the D2Q9
//   weights factor as w(c_x) w(c_y) (2/3 for 0, 1/6 for +-1), so each moment is a 1D x-stencil
//   of P*, V* (lane shifts) followed by a 1D y-stencil (rows held in registers)
//   Lambda^{n-1} = (rho~, 3 u~ + 9 s~.u - 3 rho~ u + 2A sum_b D_b^T s~_ab)
// Every lane that a needed P* sits on has both neighbours inside the wave, so the boundary
// seeds of column-adjacent faces come from lane shifts as well.
constexpr int SWA = 58;  // output columns per adjoint wave strip
constexpr int RGA = 2;   // output rows of a general unit (faces, wraps)

template <typename T, bool IN, int NR>
__device__ __forceinline__ void adj2d_rows(const AdjArgs<T> &a, int strip, int y0) {
    constexpr int H = IN ? 1 : 2;          // moment rows beyond the outputs (strain transpose)
    constexpr int NM = NR + 2 * H;         // moment rows y0 - H ..
    constexpr int NP = NM + 2;             // P*, V* rows y0 - H - 1 ..
    constexpr int NL = IN ? NP : NP + 2;   // lambda rows (one more each side for boundary seeds)
    constexpr int LOFF = IN ? 0 : 1;       // lambda row of P* row 0
    const int lane = threadIdx.x & 63;
    const Geom &g = a.g;
    const int nx = g.n[0], ny = g.n[1];
    const int c = strip * SWA - 3 + lane;
    int cw = c;
    const bool cin = IN || wrapc(cw, nx, g.per[0]);
    const int yp0 = y0 - H - 1, yl0 = yp0 - LOFF;
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const bool kobj = obj_on && obj_uses_kappa(a.obj.kind);
    const double sc = a.obj.scale;
    const int cmin = strip * SWA - 3;
    const bool wbox = a.m.hi[0] >= cmin && a.m.lo[0] <= cmin + 63 && a.m.hi[1] >= yl0 &&
                      a.m.lo[1] <= yl0 + NL - 1;
    const bool brink = wbox || a.kstatic != nullptr;

    // ---- lambda rows (and kappa, u_S where the footprint box meets the wave) ----
    // loads are unconditional from clamped indices (element 0 where a node is off the domain or
    // off the box) and select zero afterwards: no load sits behind a per-lane branch, so the wait
    // counters can follow each one
    T lp[NL], lx[NL], ly[NL], kk[NL], ksx[NL], ksy[NL];
    bool lv[NL];
    const LKS_GLOBAL T *__restrict__ Pin = gld(a.Pin);
    const LKS_GLOBAL T *__restrict__ Vin0 = gld(a.Vin[0]);
    const LKS_GLOBAL T *__restrict__ Vin1 = gld(a.Vin[1]);
#pragma unroll
    for (int k = 0; k < NL; ++k) {
        int rw = yl0 + k;
        lv[k] = cin && (IN || wrapc(rw, ny, g.per[1]));
        const long long idx = lv[k] ? cw + (long long)rw * g.sy : 0;
        const T p0 = Pin[idx], v0 = Vin0[idx], v1 = Vin1[idx];
        lp[k] = lv[k] ? p0 : T(0);
        lx[k] = lv[k] ? v0 : T(0);
        ly[k] = lv[k] ? v1 : T(0);
        kk[k] = ksx[k] = ksy[k] = T(0);
    }
    // velocities the outputs and kappa_bar need, requested with the lambda rows
    const bool out_lane = lane >= 3 && lane <= 60 && c < nx;
    T upx[NR], upy[NR], ucx[NR], ucy[NR];
#pragma unroll
    for (int ko = 0; ko < NR; ++ko) {
        const int o = y0 + ko;
        const bool ok = out_lane && o < ny;
        const long long idx = ok ? c + (long long)o * g.sy : 0;
        const T p0 = gld(a.uprev[0])[idx], p1 = gld(a.uprev[1])[idx];
        upx[ko] = ok ? p0 : T(0);
        upy[ko] = ok ? p1 : T(0);
        ucx[ko] = ucy[ko] = T(0);
    }
    // kappa, u_S and u^n on the footprint, in one block after the rows above: indices from
    // clamped coordinates (no per-lane branch), every load issued before the first select
    if (wbox) {  // wave-uniform
        T k0[NL], s0[NL], s1[NL], c0[NR], c1[NR];
        int rws[NL];
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            int rw = yl0 + k;
            if (!IN) wrapc(rw, ny, g.per[1]);
            rws[k] = rw;
            const int bi = box_index2_clamped(a.box, a.m, cw, rw);
            k0[k] = gld(a.kbox)[bi];
            s0[k] = gld(a.usbox[0])[bi];
            s1[k] = gld(a.usbox[1])[bi];
        }
#pragma unroll
        for (int ko = 0; ko < NR; ++ko) {
            const int o = min(y0 + ko, ny - 1);
            const int cx = min(max(c, a.m.lo[0]), a.m.hi[0]), oy = min(max(o, a.m.lo[1]), a.m.hi[1]);
            const long long ib = cx + (long long)oy * g.sy;  // a node of the box: inside the grid
            c0[ko] = gld(a.ucur[0])[ib];
            c1[ko] = gld(a.ucur[1])[ib];
        }
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            const bool inb = lv[k] && in_box(a.m, 2, cw, rws[k], 0);
            kk[k] = inb ? k0[k] : T(0);
            ksx[k] = inb ? s0[k] : T(0);
            ksy[k] = inb ? s1[k] : T(0);
        }
#pragma unroll
        for (int ko = 0; ko < NR; ++ko) {
            const int o = y0 + ko;
            const bool okb = out_lane && o < ny && in_box(a.m, 2, c, o, 0);
            ucx[ko] = okb ? c0[ko] : T(0);
            ucy[ko] = okb ? c1[ko] : T(0);
        }
    }
    if (obj_on && (wbox || !kobj)) {  // kappa objectives are non-zero on the footprint only
#pragma unroll
        for (int k = 0; k < NL; ++k) {
            int rw = yl0 + k;
            if (!lv[k]) continue;
            if (!IN) wrapc(rw, ny, g.per[1]);
            const long long idx = cw + (long long)rw * g.sy;
            if (a.obj.mask && !gld(a.obj.mask)[idx]) continue;
            if (kobj && kk[k] == T(0)) continue;  // kappa objectives vanish off the body
            const double us[3] = {(double)ksx[k], (double)ksy[k], 0.0};
            double dP, dV[3];
            obj_dstate(a.obj, cw, rw, 0, (double)kk[k], us, dP, dV);
            lp[k] += (T)(sc * dP);
            lx[k] += (T)(sc * dV[0]);
            ly[k] += (T)(sc * dV[1]);
        }
    }

    // ---- (P*, V*): boundary transpose and force transpose; kappa_bar on own nodes ----
    T pp[NP], px[NP], py[NP];
    const bool xadj = !IN && !g.per[0] && (cmin <= 1 || cmin + 63 >= nx - 2);  // seeds via lane shifts
#pragma unroll
    for (int kp = 0; kp < NP; ++kp) {
        const int k = kp + LOFF;
        int rw = yp0 + kp;
        T P = lp[k], Vx = lx[k], Vy = ly[k];
        if (!IN) {
            // shifted lambda of rows k-1..k+1 (every lane runs the shifts)
            T sL[3][3], sR[3][3];
            if (xadj) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    const int kd = k - 1 + d;
                    sL[d][0] = from_left(lp[kd]); sR[d][0] = from_right(lp[kd]);
                    sL[d][1] = from_left(lx[kd]); sR[d][1] = from_right(lx[kd]);
                    sL[d][2] = from_left(ly[kd]); sR[d][2] = from_right(ly[kd]);
                }
            }
            const bool rin = wrapc(rw, ny, g.per[1]);
            if (lv[k] && rin && !on_face(g, 0, cw) && !on_face(g, 1, rw)) {
                T acc[4] = {P, Vx, Vy, T(0)};
                const int c3[3] = {cw, rw, 0};
                gather_boundary_T<2>(g, a.bc.kind, c3, acc, [&](const int p[3], int comp) -> T {
                    const int dy = p[1] - rw, dx = p[0] - cw;
                    T v0, vm, vp;  // rows k-1, k, k+1 at column p[0]
                    if (dx == 0) {
                        v0 = comp == 0 ? lp[k] : comp == 1 ? lx[k] : ly[k];
                        vm = comp == 0 ? lp[k - 1] : comp == 1 ? lx[k - 1] : ly[k - 1];
                        vp = comp == 0 ? lp[k + 1] : comp == 1 ? lx[k + 1] : ly[k + 1];
                    } else {
                        const T(*sh)[3] = dx < 0 ? sL : sR;
                        v0 = sh[1][comp];
                        vm = sh[0][comp];
                        vp = sh[2][comp];
                    }
                    return dy == 0 ? v0 : dy < 0 ? vm : vp;
                });
                P = acc[0];
                Vx = acc[1];
                Vy = acc[2];
            } else {
                P = Vx = Vy = T(0);
            }
        }
        if (brink) {  // rw is wrapped here whenever lv[k] holds
            const T ks = (a.kstatic && lv[k]) ? gld(a.kstatic)[cw + (long long)rw * g.sy] : T(0);
            const T inv = rcp_t(T(1) + kk[k] + ks);
            Vx *= inv;
            Vy *= inv;
        }
        pp[kp] = P;
        px[kp] = Vx;
        py[kp] = Vy;
        // kappa_bar on the wave's own nodes of the footprint box
        const int o = yp0 + kp;
        if (wbox && kp >= H + 1 && kp < H + 1 + NR && out_lane && o < ny && in_box(a.m, 2, c, o, 0)) {
            const long long idx = c + (long long)o * g.sy;
            const long long bi = box_index(a.box, a.m, 2, c, o, 0);
            const T ux = ucx[kp - H - 1], uy = ucy[kp - H - 1];
            double kb = -((double)Vx * ((double)ux - (double)ksx[k]) + (double)Vy * ((double)uy - (double)ksy[k]));
            if (kobj && (!a.obj.mask || gld(a.obj.mask)[idx])) {
                const double uu[3] = {(double)ux, (double)uy, 0.0};
                const double uss[3] = {(double)ksx[k], (double)ksy[k], 0.0};
                kb += sc * obj_dkappa(a.obj, c, o, 0, uu, uss);
            }
            gst(a.kbar)[bi] = (T)kb;
        }
    }

    // ---- x-stencils of each P* row: a0 = M0 P + M1 Vx, a1 = M1 P + M2 Vx, a2 = M2 P + M1 Vx,
    //      b_j = M_j Vy, with M0 f = 2/3 f + 1/6 (f+ + f-), M1 f = 1/6 (f+ - f-), M2 f = 1/6 (f+ + f-)
    const T s6 = T(1) / T(6), t3 = T(2) / T(3);
    T xa0[NP], xa1[NP], xa2[NP], xb0[NP], xb1[NP], xb2[NP];
#pragma unroll
    for (int kp = 0; kp < NP; ++kp) {
        const T pl = from_left(pp[kp]), pr = from_right(pp[kp]);
        const T vxl = from_left(px[kp]), vxr = from_right(px[kp]);
        const T vyl = from_left(py[kp]), vyr = from_right(py[kp]);
        const T m0p = t3 * pp[kp] + s6 * (pr + pl), m1p = s6 * (pr - pl), m2p = s6 * (pr + pl);
        const T m1x = s6 * (vxr - vxl), m2x = s6 * (vxr + vxl);
        xa0[kp] = m0p + m1x;
        xa1[kp] = m1p + m2x;
        xa2[kp] = m2p + m1x;
        xb0[kp] = t3 * py[kp] + s6 * (vyr + vyl);
        xb1[kp] = s6 * (vyr - vyl);
        xb2[kp] = s6 * (vyr + vyl);
    }
    // ---- y-stencils: moment rows (P* rows km, km + 1, km + 2 = y - 1, y, y + 1) ----
    T mr[NM], mux[NM], muy[NM], mxx[NM], mxy[NM], myy[NM];
#pragma unroll
    for (int km = 0; km < NM; ++km) {
        const int j = km + 1;
        const T sa0 = xa0[j + 1] + xa0[j - 1], da0 = xa0[j + 1] - xa0[j - 1];
        const T sa1 = xa1[j + 1] + xa1[j - 1], da1 = xa1[j + 1] - xa1[j - 1];
        const T sa2 = xa2[j + 1] + xa2[j - 1];
        const T sb0 = xb0[j + 1] + xb0[j - 1], db0 = xb0[j + 1] - xb0[j - 1];
        const T sb1 = xb1[j + 1] + xb1[j - 1], db1 = xb1[j + 1] - xb1[j - 1];
        const T db2 = xb2[j + 1] - xb2[j - 1];
        myy[km] = s6 * (sa0 + db0);
        mr[km] = t3 * xa0[j] + myy[km];
        mux[km] = t3 * xa1[j] + s6 * (sa1 + db1);
        mxx[km] = t3 * xa2[j] + s6 * (sa2 + db2);
        muy[km] = s6 * (da0 + sb0);
        mxy[km] = s6 * (da1 + sb1);
    }

    // ---- Lambda^{n-1} on the output rows ----
    const T A2 = T(2) * a.A;
#pragma unroll
    for (int ko = 0; ko < NR; ++ko) {
        const int km = ko + H;
        const int o = y0 + ko;
        // x shifts of the strain moments (every lane)
        const T xxl = from_left(mxx[km]), xxr = from_right(mxx[km]);
        const T xyl = from_left(mxy[km]), xyr = from_right(mxy[km]);
        T dxx, dxy, dyxy, dyyy;
        if (IN) {
            dxx = T(0.5) * (xxl - xxr);
            dxy = T(0.5) * (xyl - xyr);
            dyxy = T(0.5) * (mxy[km - 1] - mxy[km + 1]);
            dyyy = T(0.5) * (myy[km - 1] - myy[km + 1]);
        } else {
            const T fxx[5] = {from_left(xxl), xxl, mxx[km], xxr, from_right(xxr)};
            const T fxy[5] = {from_left(xyl), xyl, mxy[km], xyr, from_right(xyr)};
            const T gxy[5] = {mxy[km - 2], mxy[km - 1], mxy[km], mxy[km + 1], mxy[km + 2]};
            const T gyy[5] = {myy[km - 2], myy[km - 1], myy[km], myy[km + 1], myy[km + 2]};
            dxx = deriv_T(fxx, c, nx, g.per[0]);
            dxy = deriv_T(fxy, c, nx, g.per[0]);
            dyxy = deriv_T(gxy, o, ny, g.per[1]);
            dyyy = deriv_T(gyy, o, ny, g.per[1]);
        }
        if (!out_lane || o >= ny) continue;
        const long long idx = c + (long long)o * g.sy;
        const T ux = upx[ko], uy = upy[ko];
        const T rt = mr[km];
        T vx = T(3) * mux[km] + T(9) * (mxx[km] * ux + mxy[km] * uy) - T(3) * rt * ux;
        T vy = T(3) * muy[km] + T(9) * (mxy[km] * ux + myy[km] * uy) - T(3) * rt * uy;
        vx += A2 * dxx;
        vx += A2 * dyxy;
        vy += A2 * dxy;
        vy += A2 * dyyy;
        gst(a.Pout)[idx] = rt;
        gst(a.Vout[0])[idx] = vx;
        gst(a.Vout[1])[idx] = vy;
    }
}

// Interior adjoint rows as one march along y.  The wave's output rows y0 .. y0 + RM - 1 need
// lambda rows y0 - 2 .. y0 + RM + 1; every one of them, and every lane's column, is at least two
// nodes from a face and needs no wrap, so there are no boundary seeds and every derivative is
// central.  lambda row r = y0 - 2 + j is requested AH rows before it is used; once it arrives it
// becomes (P*, V*) and its x-stencils, which complete moment row r - 1 (three stencil rows), which
// completes output row r - 2 (three moment rows).  Each row is loaded and transposed once.
// XF: the same march for a strip that holds an x face (x not periodic, rows as above).  Its rows
// meet no y face and wrap nowhere, so the boundary transpose reduces to the single x face: a
// face node's seed passes to the node next to it (one lane shift, per component as the face's
// rule copies it), face nodes and columns off the grid hold P* = V* = 0, and the transposed
// strain uses the one-sided coefficients of the columns next to the face.
#ifndef LKS_ADJ2D_AHEAD
#define LKS_ADJ2D_AHEAD 3
#endif
template <typename T, int RM, bool WB, bool XF>
__device__ __forceinline__ void adj2d_march(const AdjArgs<T> &a, int strip, int y0) {
    constexpr int NJ = RM + 4;
    constexpr int AH = LKS_ADJ2D_AHEAD;
    const int lane = threadIdx.x & 63;
    const Geom &g = a.g;
    const int nx = g.n[0];
    const int sy = (int)g.sy;  // grids hold fewer than 2^31 nodes
    const int cr = strip * SWA - 3 + lane;      // this lane's column
    const int c = XF ? min(max(cr, 0), nx - 1) : cr;  // column it loads from (inside the grid)
    const bool cval = !XF || cr == c;              // the lane holds a grid column
    const bool out_lane = lane >= 3 && lane <= 60 && (!XF || cr < nx);
    // x face: lane next to a face takes that face's seeds, per component as its rule copies them
    const bool nl = XF && cr == 1, nr = XF && cr == nx - 2, cface = XF && (cr == 0 || cr == nx - 1);
    const int kl = a.g.per[0] ? 0 : a.bc.kind[0], kr = a.g.per[0] ? 0 : a.bc.kind[1];
    const bool sl0 = nl && bc_copies(kl, 0, 0), sl1 = nl && bc_copies(kl, 1, 0), sl2 = nl && bc_copies(kl, 2, 0);
    const bool sr0 = nr && bc_copies(kr, 0, 0), sr1 = nr && bc_copies(kr, 1, 0), sr2 = nr && bc_copies(kr, 2, 0);
    // transposed x-derivative at this column: sum over o of D[c + o][c] f(c + o), o = -2 .. 2
    T dco[5];
    if (XF) {
        const T fz[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int o = 0; o < 5; ++o) {
            T f[5] = {fz[0], fz[1], fz[2], fz[3], fz[4]};
            f[o] = T(1);
            dco[o] = deriv_T(f, cr, nx, 0);
        }
    }
    const bool obj_on = a.obj.active && a.obj.kind != OBJ_NONE;
    const bool kobj = obj_on && obj_uses_kappa(a.obj.kind);
    const bool seeds = obj_on && (WB || !kobj);  // kappa objectives vanish off the footprint
    const T scT = (T)a.obj.scale;
    const LKS_GLOBAL T *__restrict__ Pin = gld(a.Pin);
    const LKS_GLOBAL T *__restrict__ Vin0 = gld(a.Vin[0]);
    const LKS_GLOBAL T *__restrict__ Vin1 = gld(a.Vin[1]);
    const LKS_GLOBAL T *__restrict__ up0 = gld(a.uprev[0]);
    const LKS_GLOBAL T *__restrict__ up1 = gld(a.uprev[1]);
    const LKS_GLOBAL T *__restrict__ kst = gld(a.kstatic);
    const LKS_GLOBAL uint8_t *__restrict__ omask = gld(a.obj.mask);
    const bool want_mask = obj_on && omask != nullptr;
    const bool brink = WB || kst != nullptr;

    // loads of lambda row j (and what the same slot carries: kappa, u_S and u^n of that row on the
    // footprint, u^{n-1} of output row j - 2), AH slots in flight
    T qp[AH], qx[AH], qy[AH], qk[AH], qs0[AH], qs1[AH], qc0[AH], qc1[AH], qu0[AH], qu1[AH], qks[AH];
    uint8_t qm[AH];
    auto issue = [&](int j) {
        const int s = j % AH;
        const int r = y0 - 2 + j;
        const int idx = c + r * sy;
        qp[s] = Pin[idx];
        qx[s] = Vin0[idx];
        qy[s] = Vin1[idx];
        if (WB) {
            const int bi = box_index2_clamped(a.box, a.m, c, r);
            qk[s] = gld(a.kbox)[bi];
            qs0[s] = gld(a.usbox[0])[bi];
            qs1[s] = gld(a.usbox[1])[bi];
            if (j >= 2 && j < RM + 2) {  // u^n of an output row, at a box node (inside the grid)
                const int cx = min(max(c, a.m.lo[0]), a.m.hi[0]), cy = min(max(r, a.m.lo[1]), a.m.hi[1]);
                const int ib = cx + cy * sy;
                qc0[s] = gld(a.ucur[0])[ib];
                qc1[s] = gld(a.ucur[1])[ib];
            }
        }
        if (j >= 4) {  // u^{n-1} of output row r - 2
            const int io = idx - 2 * sy;
            qu0[s] = up0[io];
            qu1[s] = up1[io];
        }
        if (kst) qks[s] = kst[idx];
        if (want_mask) qm[s] = omask[idx];
    };

    const T s6 = T(1) / T(6), t3 = T(2) / T(3);
    const T A2 = T(2) * a.A;
    T xs[3][6];   // x-stencil rows (a0, a1, a2, b0, b1, b2), ring by row
    T mo[3][6];   // moment rows (rho~, u~x, u~y, s~xx, s~xy, s~yy), ring by row
#pragma unroll
    for (int j = 0; j < AH && j < NJ; ++j) issue(j);
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int s = j % AH;
        const int r = y0 - 2 + j;
        T P = cval ? qp[s] : T(0), Vx = cval ? qx[s] : T(0), Vy = cval ? qy[s] : T(0);
        const bool inb = WB && in_box(a.m, 2, c, r, 0);
        const T kap = inb ? qk[s] : T(0), usx = inb ? qs0[s] : T(0), usy = inb ? qs1[s] : T(0);
        const T ucx = inb ? qc0[s] : T(0), ucy = inb ? qc1[s] : T(0);
        const T upx = qu0[s], upy = qu1[s];
        const T ks = kst ? qks[s] : T(0);
        const bool mk = want_mask ? qm[s] != 0 : true;
        if (j + AH < NJ) issue(j + AH);

        // lambda + dj/dX (in the path's precision), then the force transpose
        if (seeds && cval && mk && !(kobj && kap == T(0))) {
            const T us[3] = {usx, usy, T(0)};
            T dP, dV[3];
            obj_dstate_r<T>(a.obj, c, r, 0, kap, us, dP, dV);
            P += scT * dP;
            Vx += scT * dV[0];
            Vy += scT * dV[1];
        }
        if (XF) {  // boundary transpose of the x face
            const T pL = from_left(P), xL = from_left(Vx), yL = from_left(Vy);
            const T pR = from_right(P), xR = from_right(Vx), yR = from_right(Vy);
            P += (sl0 ? pL : T(0)) + (sr0 ? pR : T(0));
            Vx += (sl1 ? xL : T(0)) + (sr1 ? xR : T(0));
            Vy += (sl2 ? yL : T(0)) + (sr2 ? yR : T(0));
            if (cface || !cval) P = Vx = Vy = T(0);
        }
        if (brink) {
            const T inv = rcp_t(T(1) + kap + ks);
            Vx *= inv;
            Vy *= inv;
        }
        // kappa_bar on the wave's own footprint nodes of its output rows
        if (WB && j >= 2 && j < RM + 2 && out_lane && inb) {
            T kb = -(Vx * (ucx - usx) + Vy * (ucy - usy));
            if (kobj && mk) {
                const T uu[3] = {ucx, ucy, T(0)}, uss[3] = {usx, usy, T(0)};
                kb += scT * obj_dkappa_r<T>(a.obj, c, r, 0, uu, uss);
            }
            gst(a.kbar)[box_index(a.box, a.m, 2, c, r, 0)] = kb;
        }

        // x-stencils of row r: a0 = M0 P + M1 Vx, a1 = M1 P + M2 Vx, a2 = M2 P + M1 Vx, b_k = M_k Vy
        {
            T *x = xs[j % 3];
            const T pl = from_left(P), pr = from_right(P);
            const T vxl = from_left(Vx), vxr = from_right(Vx);
            const T vyl = from_left(Vy), vyr = from_right(Vy);
            const T m0p = t3 * P + s6 * (pr + pl), m1p = s6 * (pr - pl), m2p = s6 * (pr + pl);
            const T m1x = s6 * (vxr - vxl), m2x = s6 * (vxr + vxl);
            x[0] = m0p + m1x;
            x[1] = m1p + m2x;
            x[2] = m2p + m1x;
            x[3] = t3 * Vy + s6 * (vyr + vyl);
            x[4] = s6 * (vyr - vyl);
            x[5] = s6 * (vyr + vyl);
        }
        // moment row r - 1 from stencil rows r - 2, r - 1, r
        if (j >= 2) {
            const T *xm = xs[(j - 2) % 3], *x0 = xs[(j - 1) % 3], *xp = xs[j % 3];
            T *m = mo[(j - 1) % 3];
            const T sa0 = xp[0] + xm[0], da0 = xp[0] - xm[0];
            const T sa1 = xp[1] + xm[1], da1 = xp[1] - xm[1];
            const T sa2 = xp[2] + xm[2];
            const T sb0 = xp[3] + xm[3], db0 = xp[3] - xm[3];
            const T sb1 = xp[4] + xm[4], db1 = xp[4] - xm[4];
            const T db2 = xp[5] - xm[5];
            m[5] = s6 * (sa0 + db0);
            m[0] = t3 * x0[0] + m[5];
            m[1] = t3 * x0[1] + s6 * (sa1 + db1);
            m[3] = t3 * x0[2] + s6 * (sa2 + db2);
            m[2] = s6 * (da0 + sb0);
            m[4] = s6 * (da1 + sb1);
        }
        // Lambda^{n-1} on output row r - 2 from moment rows r - 3, r - 2, r - 1
        if (j >= 4) {
            const T *mm = mo[(j - 3) % 3], *m0 = mo[(j - 2) % 3], *mp = mo[(j - 1) % 3];
            const T xxl = from_left(m0[3]), xxr = from_right(m0[3]);
            const T xyl = from_left(m0[4]), xyr = from_right(m0[4]);
            T dxx, dxy;
            if (XF) {
                dxx = dco[0] * from_left(xxl) + dco[1] * xxl + dco[2] * m0[3] + dco[3] * xxr + dco[4] * from_right(xxr);
                dxy = dco[0] * from_left(xyl) + dco[1] * xyl + dco[2] * m0[4] + dco[3] * xyr + dco[4] * from_right(xyr);
            } else {
                dxx = T(0.5) * (xxl - xxr);
                dxy = T(0.5) * (xyl - xyr);
            }
            const T dyxy = T(0.5) * (mm[4] - mp[4]);
            const T dyyy = T(0.5) * (mm[5] - mp[5]);
            const T rt = m0[0];
            T vx = T(3) * m0[1] + T(9) * (m0[3] * upx + m0[4] * upy) - T(3) * rt * upx;
            T vy = T(3) * m0[2] + T(9) * (m0[4] * upx + m0[5] * upy) - T(3) * rt * upy;
            vx += A2 * dxx;
            vx += A2 * dyxy;
            vy += A2 * dxy;
            vy += A2 * dyyy;
            if (out_lane) {
                const int io = c + (r - 2) * sy;
                gst(a.Pout)[io] = rt;
                gst(a.Vout[0])[io] = vx;
                gst(a.Vout[1])[io] = vy;
            }
        }
    }
}

// Work units of one 2D adjoint step, one per wave.  Over rows [4, yhi), in chunks of RMA rows,
// every strip marches: inner strips (every lane's column at least one node off the x faces, no
// wrap) with the interior variant, the outer strips that hold an x face with the XF variant (x not
// periodic).  Everything else — the four rows next to each y face (or the wrap of a periodic y),
// and all rows of the outer strips when x is periodic — is a general unit of RGA rows with the
// full boundary transpose.  March units come first (they are the longest), then the outer strips'
// general units, then the y-edge units of the marching strips.  Six rows per march: the launch
// alone is faster at eight (14.0 against 14.9 us at 1024^2), but the reverse sweep, where the
// segment recompute shares the GPU, is faster at six (1024^2 D2Q9, 10^4 steps, checkpoint every
// 100: 36.7 k -> 36.9 k MLUPS; 4, 5 and 10 rows slower).
#ifndef LKS_ADJ2D_RM
#define LKS_ADJ2D_RM 6
#endif
constexpr int RMA = LKS_ADJ2D_RM;
struct Adj2dUnits {
    int nstrips, ninner, nms, nmc, yhi, ngs, ngr, neg;
    long long nmarch, nouter, total;
};
__host__ __device__ inline Adj2dUnits adj2d_units(const Geom &g) {
    Adj2dUnits u;
    const int nx = g.n[0], ny = g.n[1];
    u.nstrips = (nx + SWA - 1) / SWA;
    u.nmc = ny >= 8 ? (ny - 8) / RMA : 0;
    u.ninner = (u.nmc > 0 && nx >= 2 * SWA + 4) ? (nx - 62) / SWA : 0;
    if (u.ninner == 0) u.nmc = 0;
    u.yhi = 4 + RMA * u.nmc;
    u.ngs = u.nstrips - u.ninner;
    u.nms = u.ninner + ((u.nmc > 0 && !g.per[0]) ? u.ngs : 0);  // marching strips
    u.ngr = (ny + RGA - 1) / RGA;
    u.neg = u.nms > 0 ? 4 + (ny - u.yhi) : 0;  // y-edge units of one row each
    u.nmarch = (long long)u.nms * u.nmc;
    u.nouter = u.nms > u.ninner ? 0 : (long long)u.ngs * u.ngr;
    u.total = u.nmarch + u.nouter + (long long)u.nms * u.neg;
    return u;
}

// strip of marching-strip index i: inner strips 1 .. ninner, then the outer ones
__host__ __device__ inline int adj2d_mstrip(const Adj2dUnits &u, int i) {
    return i < u.ninner ? 1 + i : (i == u.ninner ? 0 : i);
}

template <typename T>
__device__ __forceinline__ void adj2d_unit(const AdjArgs<T> &a, const Adj2dUnits &u, long long k) {
    int strip, y0;
    if (k < u.nmarch) {
        const int kk = (int)k, i = kk % u.nms;
        strip = adj2d_mstrip(u, i);
        y0 = 4 + RMA * (kk / u.nms);
        const int cmin = strip * SWA - 3;
        const bool wbox = a.m.hi[0] >= cmin && a.m.lo[0] <= cmin + 63 && a.m.hi[1] >= y0 - 2 &&
                          a.m.lo[1] <= y0 + RMA + 1;
        if (i < u.ninner) {
            if (wbox) adj2d_march<T, RMA, true, false>(a, strip, y0);
            else adj2d_march<T, RMA, false, false>(a, strip, y0);
        } else {
            if (wbox) adj2d_march<T, RMA, true, true>(a, strip, y0);
            else adj2d_march<T, RMA, false, true>(a, strip, y0);
        }
        return;
    }
    if (k < u.nmarch + u.nouter) {
        const int v = (int)(k - u.nmarch);
        const int q = v % u.ngs;
        strip = q == 0 ? 0 : u.ninner + q;
        y0 = RGA * (v / u.ngs);
    } else {
        const int v = (int)(k - u.nmarch - u.nouter);
        const int q = v / u.nms;
        strip = adj2d_mstrip(u, v % u.nms);
        y0 = q < 4 ? q : u.yhi + (q - 4);
        adj2d_rows<T, false, 1>(a, strip, y0);  // one row: these general units finish with the marches
        return;
    }
    adj2d_rows<T, false, RGA>(a, strip, y0);
}

#ifndef LKS_ADJ2D_WAVES
#define LKS_ADJ2D_WAVES 1
#endif
// the second bound asks for that many resident waves per SIMD (register budget)
template <typename T>
__global__ __launch_bounds__(kBlock, LKS_ADJ2D_WAVES) void k_adj2d_batch(const AdjArgs<T> *__restrict__ args,
                                                                         const long long *__restrict__ tile0,
                                                                         int njobs) {
    const long long b = blockIdx.x;
    const int j = __builtin_amdgcn_readfirstlane(job_of(tile0, njobs, b));
    const AdjArgs<T> &a = args[j];
    touch_lines<sizeof(AdjArgs<T>)>(&a);
    const long long t = njobs == 1 ? b : b - tile0[j];  // one job: tile0 = {0}
    const Adj2dUnits u = adj2d_units(a.g);
    const long long na = (u.total + WPB - 1) / WPB;
    if (t >= na) {  // extra blocks: sensitivity gather of the previous adjoint step
        sens_body<T>(*a.sens, t - na);
        return;
    }
    const long long k = t * WPB + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (k < u.total) adj2d_unit<T>(a, u, k);
    prefetch_next<sizeof(AdjArgs<T>)>(a.next);
}

long long fwd_blocks(const Geom &g, int lattice, int esz) {
    // one objective partial per wave (2D) or per block (3D)
    if (g.dim == 2) return fwd2d_nblocks(g) * WPB;
    return fwd_blocks3d(g, lattice, esz);
}

long long xfer_blocks(int dim, long long cells, int esz) {
    if (dim == 2) return (cells + kBlock - 1) / kBlock;
    return xfer_blocks3d(cells, esz);
}

long long tiles2d_fwd(const Geom &g) { return fwd2d_nblocks(g); }
long long tiles2d(const Geom &g) { return (adj2d_units(g).total + WPB - 1) / WPB; }

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

// The paper's own adjoint step (Sec. 2.4, Eqs. arho, au, as, the adjoint equilibrium and the
// source-term updates arho_ex, au_ex, as_ex), 2D: the variant of the exact reverse step in which
// (i) the Brinkman source divides only the pulled velocity moment 3 u~ (with the objective's u-seed)
// by (1 + kappa), and (ii) the kappa seed is formed from that moment alone:
//   kappa_bar = -(3 u~ / (1 + kappa)) . (u - u_S) + dj/dkappa.
// Everything else (objective seeds, boundary transposes, the pull from x + c_i, the w-moments and
// the transposed equilibrium and strain) is the exact step's.  Three plain launches per step, one
// thread per node (the variant serves verification, not throughput):
//   prep     lambda + seeds, boundary transpose, paper force transpose -> (P*, V*), kappa_bar
//   moments  pull of E~_i(y) = P*(y + c_i) + c_i . V*(y + c_i), w-moments rho~, u~, s~ ->
//            P = rho~, U3 = 3 u~, V = 3 u~ + 9 s~ u - 3 rho~ u; s~ kept for the next launch
//   strain   V += the transposed strain operator applied to A (s~ + s~^T) (gather form)
#include "lks_device.hpp"

namespace lks {

namespace {

template <typename T>
__device__ __forceinline__ bool node_of(const Geom &g, long long t, int &x, int &y) {
    if (t >= (long long)g.n[0] * g.n[1]) return false;
    const unsigned tu = (unsigned)t, n0 = (unsigned)g.n[0];  // fewer than 2^31 nodes
    x = (int)(tu % n0);
    y = (int)(tu / n0);
    return true;
}

// lambda of node (x, y) plus its objective seeds (u-seed returned separately in su[2])
template <typename T>
__device__ void seeded_lambda(const AdjArgs<T> &a, int x, int y, T l[3], T su[2], T &kap, T us[2]) {
    const Geom &g = a.g;
    const long long idx = x + (long long)y * g.sy;
    l[0] = a.Pin[idx];
    l[1] = a.Vin[0][idx];
    l[2] = a.Vin[1][idx];
    su[0] = su[1] = T(0);
    kap = T(0);
    us[0] = us[1] = T(0);
    if (in_box(a.m, 2, x, y, 0)) {
        const long long bi = box_index(a.box, a.m, 2, x, y, 0);
        kap = a.kbox[bi];
        us[0] = a.usbox[0][bi];
        us[1] = a.usbox[1][bi];
    }
    if (a.obj.active && (!a.obj.mask || a.obj.mask[idx])) {
        const double uss[3] = {(double)us[0], (double)us[1], 0.0};
        double dP, dV[3];
        obj_dstate(a.obj, x, y, 0, (double)kap, uss, dP, dV);
        const double sc = a.obj.scale;
        l[0] += (T)(sc * dP);
        su[0] = (T)(sc * dV[0]);
        su[1] = (T)(sc * dV[1]);
        l[1] += su[0];
        l[2] += su[1];
    }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kBlock) void k_padj2d_prep(const AdjArgs<T> *__restrict__ args) {
    const AdjArgs<T> &a = args[0];
    const Geom &g = a.g;
    int x, y;
    if (!node_of<T>(g, blockIdx.x * (long long)kBlock + threadIdx.x, x, y)) return;
    const long long idx = x + (long long)y * g.sy;
    if (on_face(g, 0, x) || on_face(g, 1, y)) {  // nothing flows through face nodes
        a.Ps[idx] = T(0);
        a.Vs[0][idx] = T(0);
        a.Vs[1][idx] = T(0);
        return;
    }
    T l[3], su[2], kap, us[2];
    seeded_lambda(a, x, y, l, su, kap, us);
    T acc[4] = {l[0], l[1], l[2], T(0)};
    const int c3[3] = {x, y, 0};
    gather_boundary_T<2>(g, a.bc.kind, c3, acc, [&](const int p[3], int comp) -> T {
        T pl[3], psu[2], pk, pus[2];
        seeded_lambda(a, p[0], p[1], pl, psu, pk, pus);
        return pl[comp];
    });
    const T ks = a.kstatic ? a.kstatic[idx] : T(0);
    const T den = T(1) + kap + ks;
    T q[2];
    for (int c = 0; c < 2; ++c) {
        const T u3 = a.U3in[c][idx] + su[c];  // Eq. au_ex: the u-seed joins u~ before the division
        q[c] = u3 / den;
        a.Vs[c][idx] = q[c] + (acc[1 + c] - u3);
    }
    a.Ps[idx] = acc[0];
    if (in_box(a.m, 2, x, y, 0)) {
        double kb = -((double)q[0] * ((double)a.ucur[0][idx] - (double)us[0]) +
                      (double)q[1] * ((double)a.ucur[1][idx] - (double)us[1]));
        if (a.obj.active && obj_uses_kappa(a.obj.kind) && (!a.obj.mask || a.obj.mask[idx])) {
            const double uu[3] = {(double)a.ucur[0][idx], (double)a.ucur[1][idx], 0.0};
            const double uss[3] = {(double)us[0], (double)us[1], 0.0};
            kb += a.obj.scale * obj_dkappa(a.obj, x, y, 0, uu, uss);
        }
        a.kbar[box_index(a.box, a.m, 2, x, y, 0)] = (T)kb;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_padj2d_moments(const AdjArgs<T> *__restrict__ args) {
    const AdjArgs<T> &a = args[0];
    const Geom &g = a.g;
    int x, y;
    if (!node_of<T>(g, blockIdx.x * (long long)kBlock + threadIdx.x, x, y)) return;
    constexpr int C[9][2] = {{0, 0}, {1, 0}, {0, 1}, {-1, 0}, {0, -1}, {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    constexpr double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
    T rt = T(0), ut[2] = {T(0), T(0)}, sxx = T(0), sxy = T(0), syy = T(0);
    for (int i = 0; i < 9; ++i) {
        int zx = x + C[i][0], zy = y + C[i][1];
        if (!wrapc(zx, g.n[0], g.per[0]) || !wrapc(zy, g.n[1], g.per[1])) continue;
        const long long zi = zx + (long long)zy * g.sy;
        const T eb = a.Ps[zi] + T(C[i][0]) * a.Vs[0][zi] + T(C[i][1]) * a.Vs[1][zi];
        const T w = (T)W[i];
        rt += w * eb;
        ut[0] += w * T(C[i][0]) * eb;
        ut[1] += w * T(C[i][1]) * eb;
        sxx += w * T(C[i][0] * C[i][0]) * eb;
        sxy += w * T(C[i][0] * C[i][1]) * eb;
        syy += w * T(C[i][1] * C[i][1]) * eb;
    }
    const long long idx = x + (long long)y * g.sy;
    const T ux = a.uprev[0][idx], uy = a.uprev[1][idx];
    a.Pout[idx] = rt;
    a.U3out[0][idx] = T(3) * ut[0];
    a.U3out[1][idx] = T(3) * ut[1];
    a.Vout[0][idx] = T(3) * ut[0] - T(3) * rt * ux + T(9) * (sxx * ux + sxy * uy);
    a.Vout[1][idx] = T(3) * ut[1] - T(3) * rt * uy + T(9) * (sxy * ux + syy * uy);
    a.st[0][idx] = sxx;
    a.st[1][idx] = sxy;
    a.st[2][idx] = syy;
}

// V_a(y) += sum_q sum_z coef_q(z -> y) A (s~_aq(z) + s~_qa(z)): z runs over the nodes whose
// difference row along q (central, or one-sided at a non-periodic face) reads node y.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_padj2d_strain(const AdjArgs<T> *__restrict__ args) {
    const AdjArgs<T> &a = args[0];
    const Geom &g = a.g;
    int x, y;
    if (!node_of<T>(g, blockIdx.x * (long long)kBlock + threadIdx.x, x, y)) return;
    const int yc[2] = {x, y};
    T add[2] = {T(0), T(0)};
    for (int q = 0; q < 2; ++q) {
        const int n = g.n[q], per = g.per[q], c = yc[q];
        auto contrib = [&](int zq, T coef) {
            int z[2] = {x, y};
            z[q] = zq;
            const long long zi = z[0] + (long long)z[1] * g.sy;
            const T s0q = q == 0 ? a.st[0][zi] : a.st[1][zi];  // s~_{x q}
            const T s1q = q == 0 ? a.st[1][zi] : a.st[2][zi];  // s~_{y q}
            add[0] += coef * a.A * (s0q + s0q);
            add[1] += coef * a.A * (s1q + s1q);
        };
        // central rows of z = y -/+ e (coef +/- 1/2 on y)
        for (int s = -1; s <= 1; s += 2) {
            int zq = c + s;
            if (!wrapc(zq, n, per)) continue;
            if (!per && (zq == 0 || zq == n - 1)) continue;  // z on a face: one-sided row
            contrib(zq, s < 0 ? T(0.5) : T(-0.5));
        }
        if (!per) {
            if (c <= 2) contrib(0, c == 0 ? T(-1.5) : c == 1 ? T(2.0) : T(-0.5));
            if (c >= n - 3) contrib(n - 1, c == n - 1 ? T(1.5) : c == n - 2 ? T(-2.0) : T(0.5));
        }
    }
    const long long idx = x + (long long)y * g.sy;
    a.Vout[0][idx] += add[0];
    a.Vout[1][idx] += add[1];
}

template <typename T>
hipError_t launch_padj2d(const AdjArgs<T> *args, const Geom &g, hipStream_t s) {
    const long long n = (long long)g.n[0] * g.n[1];
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock));
    hipLaunchKernelGGL(k_padj2d_prep<T>, grid, dim3(kBlock), 0, s, args);
    hipLaunchKernelGGL(k_padj2d_moments<T>, grid, dim3(kBlock), 0, s, args);
    hipLaunchKernelGGL(k_padj2d_strain<T>, grid, dim3(kBlock), 0, s, args);
    return hipGetLastError();
}

template hipError_t launch_padj2d<float>(const AdjArgs<float> *, const Geom &, hipStream_t);
template hipError_t launch_padj2d<double>(const AdjArgs<double> *, const Geom &, hipStream_t);

}  // namespace lks

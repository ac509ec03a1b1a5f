// Host runtime of the LKS library: descriptor validation, the HBM ledger, device buffers, and
// the drivers of Algorithm 1 (forward with state checkpoints every K steps) and of the reverse
// sweep (restore a checkpoint, recompute its segment into the trajectory store, then run the
// adjoint step and the sensitivity gather for each step of the segment, last step first).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lks.h"
#include "lks_internal.hpp"

namespace lks {
constexpr long long kBlockHost = 256;  // threads per block of the pointwise kernels
}
using lks::BoxGeom;
using lks::Geom;
using lks::StepMotion;

namespace {

thread_local std::string g_create_error;
constexpr int kPartialRows = 64;

const char *kind_name(int k) {
    switch (k) {
    case 0: return "forward step";
    case 1: return "adjoint step";
    case 2: return "sensitivity gather";
    }
    return "?";
}

struct Layout {
    Geom g{};
    long long pitch = 0;     // padded row length (elements)
    long long F = 0;         // elements per field
    long long ncell = 0;
    long long nd = 0;
    int K = 0;               // segment length
    int S = 0;               // number of segments (= checkpoints)
    size_t esz = 0;
    BoxGeom box{};
    std::vector<StepMotion> steps;  // index n = 0..N
    size_t bytes = 0;
    // byte sizes of each allocation
    size_t b_state = 0, b_ckpt = 0, b_traj = 0, b_box = 0, b_kbar = 0, b_adj = 0, b_design = 0,
           b_aux = 0, b_final = 0, b_pv = 0, b_args = 0, b_xring = 0, b_padj = 0;
    long long max_blocks = 0;
    int prow = 1;            // rows of the objective-partials ring (steps reduced per batch)
    int banks = 1;           // trajectory/box store banks: 2 lets a segment be recomputed while
                             // the adjoint of the following one runs
    bool fwd_only = false;   // objective NONE: forward sweep only, no trajectory or adjoint storage
};

int fail(std::string *err, int code, const std::string &msg) {
    if (err) *err = msg;
    return code;
}

bool finite3(const double *v) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

// Validate the descriptor and compute every size the context needs (no GPU call).
int plan(const lks_desc *d, Layout &L, std::string *err) {
    if (!d) return fail(err, LKS_EINVAL, "descriptor is NULL");
    if (d->dim != 2 && d->dim != 3) return fail(err, LKS_EINVAL, "dim must be 2 or 3");
    const int D = d->dim;
    if (D == 2 && d->lattice != LKS_D2Q9) return fail(err, LKS_EINVAL, "2D needs LKS_D2Q9");
    if (D == 3 && d->lattice != LKS_D3Q15 && d->lattice != LKS_D3Q19)
        return fail(err, LKS_EINVAL, "3D needs LKS_D3Q15 or LKS_D3Q19");
    if (d->precision != LKS_F32 && d->precision != LKS_F64)
        return fail(err, LKS_EINVAL, "precision must be LKS_F32 or LKS_F64");
    if (d->interp != LKS_INTERP_PAPER && d->interp != LKS_INTERP_FLUID_ONE)
        return fail(err, LKS_EINVAL, "unknown interpolation");
    if (d->weight != LKS_W_COS4 && d->weight != LKS_W_LIN)
        return fail(err, LKS_EINVAL, "unknown transfer weight");
    if (!(d->nu > 0.0) || !std::isfinite(d->nu)) return fail(err, LKS_EINVAL, "nu must be > 0");
    if (!(d->q > 0.0) || !std::isfinite(d->q) || !std::isfinite(d->kappa_max) || d->kappa_max < 0)
        return fail(err, LKS_EINVAL, "need q > 0 and kappa_max >= 0");
    if (d->nsteps < 1) return fail(err, LKS_EINVAL, "nsteps must be >= 1");
    if (!d->motion) return fail(err, LKS_EINVAL, "motion table is NULL");
    if (d->checkpoint_every < 0) return fail(err, LKS_EINVAL, "checkpoint_every must be >= 0");
    if (d->adjoint_form != LKS_ADJ_EXACT && d->adjoint_form != LKS_ADJ_PAPER)
        return fail(err, LKS_EINVAL, "unknown adjoint form");
    if (d->adjoint_form == LKS_ADJ_PAPER && d->dim != 2)
        return fail(err, LKS_EUNSUPPORTED, "the paper's adjoint form is built for 2D");
    if (d->zchunk != 0 && (d->zchunk < 8 || d->zchunk > 32))
        return fail(err, LKS_EINVAL, "zchunk must be 0 or in [8, 32]");
    if (!std::isfinite(d->rho0) || !finite3(d->u0) || !finite3(d->body_force) || !finite3(d->xi_G))
        return fail(err, LKS_EINVAL, "non-finite initial state, force or xi_G");

    Geom &g = L.g;
    g.dim = D;
    for (int a = 0; a < 3; ++a) {
        if (a >= D) {
            if (d->n[a] != 1 || d->nd[a] != 1) return fail(err, LKS_EINVAL, "2D needs n[2] = nd[2] = 1");
            g.n[a] = 1;
            g.per[a] = 1;
            continue;
        }
        const int km = d->bc[2 * a].kind, kp = d->bc[2 * a + 1].kind;
        for (int k : {km, kp})
            if (k < LKS_BC_PERIODIC || k > LKS_BC_NOSLIP) return fail(err, LKS_EINVAL, "unknown boundary kind");
        if ((km == LKS_BC_PERIODIC) != (kp == LKS_BC_PERIODIC))
            return fail(err, LKS_EINVAL, "both faces of a periodic axis must be PERIODIC");
        g.per[a] = km == LKS_BC_PERIODIC;
        if (d->n[a] < (g.per[a] ? 3 : 4))
            return fail(err, LKS_EINVAL, "n must be >= 4 on non-periodic axes and >= 3 on periodic ones");
        if (d->n[a] > (1 << 20) || d->nd[a] < 1 || d->nd[a] > (1 << 20))
            return fail(err, LKS_EINVAL, "grid extent out of range");
        g.n[a] = d->n[a];
        for (int s = 0; s < 2; ++s) {
            const lks_bc &bf = d->bc[2 * a + s];
            if (!std::isfinite(bf.rho) || !finite3(bf.u))
                return fail(err, LKS_EINVAL, "non-finite boundary value");
            if ((bf.kind == LKS_BC_PRESSURE || bf.kind == LKS_BC_ZERO_GRADIENT) && !(bf.rho > 0.0))
                return fail(err, LKS_EINVAL, "PRESSURE and ZERO_GRADIENT faces need rho_bar > 0");
        }
    }
    const lks_objective &ob = d->objective;
    if (ob.kind != LKS_OBJ_NONE) {
        if (ob.kind < LKS_OBJ_POWER || ob.kind > LKS_OBJ_MASS) return fail(err, LKS_EINVAL, "unknown objective");
        if (ob.n0 < 1 || ob.n1 > d->nsteps || ob.n0 > ob.n1)
            return fail(err, LKS_EINVAL, "objective window must satisfy 1 <= n0 <= n1 <= nsteps");
        if (!finite3(ob.centre) || !finite3(ob.dir)) return fail(err, LKS_EINVAL, "non-finite objective vector");
    }

    L.pitch = ((g.n[0] + 63) / 64) * 64;
    g.sy = L.pitch;
    g.sz = L.pitch * g.n[1];
    L.F = g.sz * g.n[2];
    L.ncell = (long long)g.n[0] * g.n[1] * g.n[2];
    L.nd = (long long)d->nd[0] * d->nd[1] * d->nd[2];
    L.esz = d->precision == LKS_F64 ? 8 : 4;
    g.zc = D == 3 ? lks::choose_zc3(g, (int)L.esz) : 1;
    if (D == 3 && d->zchunk > 0) {  // the caller's chunk, evened out over the chunks of n_z
        const int nch = (g.n[2] + d->zchunk - 1) / d->zchunk;
        g.zc = (g.n[2] + nch - 1) / nch;
    }
    g.zca = D == 3 ? lks::choose_zca3(g, (int)L.esz) : 1;
    const int N = d->nsteps;
    L.fwd_only = d->objective.kind == LKS_OBJ_NONE;  // nothing to differentiate: no reverse buffers
    L.K = (L.fwd_only || d->checkpoint_every == 0 || d->checkpoint_every >= N) ? N : d->checkpoint_every;
    L.S = (N + L.K - 1) / L.K;
    L.banks = (!L.fwd_only && L.S > 1) ? 2 : 1;

    // rigid motion: orthogonal R; 2D motion stays in the plane; footprint inside the domain
    const double s = d->weight == LKS_W_LIN ? 1.0 : 2.0;
    L.steps.resize(N + 1);
    int bn[3] = {1, 1, 1};
    for (int n = 0; n <= N; ++n) {
        const lks_motion &m = d->motion[n];
        for (int i = 0; i < 9; ++i)
            if (!std::isfinite(m.R[i])) return fail(err, LKS_EINVAL, "non-finite rotation");
        if (!finite3(m.omega) || !finite3(m.xG) || !finite3(m.uG))
            return fail(err, LKS_EINVAL, "non-finite motion record");
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double v = 0;
                for (int k = 0; k < 3; ++k) v += m.R[3 * i + k] * m.R[3 * j + k];
                if (std::fabs(v - (i == j ? 1.0 : 0.0)) > 1e-9)
                    return fail(err, LKS_EINVAL, "motion R is not orthogonal at step " + std::to_string(n));
            }
        if (D == 2 && (m.R[2] != 0 || m.R[5] != 0 || m.R[6] != 0 || m.R[7] != 0 || m.R[8] != 1 ||
                       m.omega[0] != 0 || m.omega[1] != 0 || m.uG[2] != 0))
            return fail(err, LKS_EINVAL, "2D motion must rotate about z and stay in the plane");
        StepMotion &sm = L.steps[n];
        std::memcpy(sm.R, m.R, sizeof sm.R);
        std::memcpy(sm.Om, m.omega, sizeof sm.Om);
        std::memcpy(sm.xG, m.xG, sizeof sm.xG);
        std::memcpy(sm.uG, m.uG, sizeof sm.uG);
        if (D == 2) sm.xG[2] = 0.0;
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (int c = 0; c < (1 << D); ++c) {
            double xi[3] = {0, 0, 0};
            for (int a = 0; a < D; ++a) xi[a] = ((c >> a) & 1) ? d->nd[a] - 1 : 0;
            for (int r = 0; r < D; ++r) {
                double v = sm.xG[r];
                for (int a = 0; a < D; ++a) v += sm.R[3 * r + a] * (xi[a] - d->xi_G[a]);
                mn[r] = std::min(mn[r], v);
                mx[r] = std::max(mx[r], v);
            }
        }
        for (int a = 0; a < 3; ++a) {
            if (a >= D) {
                sm.lo[a] = sm.hi[a] = 0;
                continue;
            }
            // nodes with a non-zero weight lie strictly inside (min - s, max + s)
            sm.lo[a] = (int)std::floor(mn[a] - s) + 1;
            sm.hi[a] = (int)std::ceil(mx[a] + s) - 1;
            const int lim_lo = g.per[a] ? 0 : 1, lim_hi = g.per[a] ? g.n[a] - 1 : g.n[a] - 2;
            if (n >= 1 && (sm.lo[a] < lim_lo || sm.hi[a] > lim_hi))
                return fail(err, LKS_EINVAL,
                            "rigid-body footprint leaves the interior at step " + std::to_string(n));
            sm.lo[a] = std::max(sm.lo[a], lim_lo);
            sm.hi[a] = std::min(sm.hi[a], lim_hi);
            bn[a] = std::max(bn[a], sm.hi[a] - sm.lo[a] + 1);
        }
    }
    L.box.bn[0] = bn[0];
    L.box.bn[1] = bn[1];
    L.box.bn[2] = bn[2];
    L.box.bsy = bn[0];
    L.box.bsz = (long long)bn[0] * bn[1];
    L.box.cells = (long long)bn[0] * bn[1] * bn[2];
    // the kernels decompose cell, design-node and box indices with 32-bit arithmetic
    if ((long long)g.n[0] * g.n[1] * g.n[2] >= (1LL << 31) || (long long)d->nd[0] * d->nd[1] * d->nd[2] >= (1LL << 31) ||
        L.box.cells >= (1LL << 31))
        return fail(err, LKS_EINVAL, "grid, design grid and footprint box must each hold fewer than 2^31 nodes");

    const size_t e = L.esz;
    const size_t nf = 1 + D;
    L.b_state = 2 * nf * L.F * e;
    L.b_ckpt = (size_t)L.S * nf * L.F * e;
    L.b_traj = L.fwd_only ? 0 : (size_t)L.banks * (L.K + 1) * D * L.F * e;
    L.b_box = L.fwd_only ? 0 : (size_t)L.banks * L.K * nf * L.box.cells * e;
    L.b_xring = 2 * nf * L.box.cells * e;  // kappa, u_S of the steps outside the stored segment
    // kappa_bar of steps n (n even / odd), padded so the gather's 5 x 5 tap windows stay in bounds
    L.b_kbar = L.fwd_only ? 0 : (size_t)(2 * L.box.cells + 4 * L.box.bsy + 8) * e;
    L.b_adj = L.fwd_only ? 0 : 2 * nf * L.F * e;
    L.b_final = nf * L.F * e;
    L.b_design = (size_t)L.nd * (3 * e + 2 * 8);  // gamma, kref, sens out; kprime, G
    L.max_blocks = lks::fwd_blocks(g, d->lattice, (int)L.esz);
    L.b_pv = (D == 3 && !L.fwd_only) ? (size_t)4 * L.F * e : 0;  // (P*, V*) between the 3D adjoint kernels
    // the paper's adjoint form: (P*, V*), 3 u~ of two levels and s~ (xx, xy, yy)
    L.b_padj = (d->adjoint_form == LKS_ADJ_PAPER && !L.fwd_only) ? (size_t)(nf + 2 * D + 3) * L.F * e : 0;
    // objective partials: a ring of rows of per-wave (2D) or per-block (3D) sums, one row per step,
    // reduced into j^n every kPartialRows steps of the window and at its end
    const long long obj_rows = d->objective.kind == LKS_OBJ_NONE ? 1 : (d->objective.n1 - d->objective.n0 + 1);
    L.prow = (int)std::min<long long>(obj_rows, kPartialRows);
    L.b_aux = (size_t)(d->nsteps + 1) * 8 + (size_t)L.prow * L.max_blocks * 8 + 64;
    if (d->kappa_static) L.b_aux += L.F * e;
    if (d->objective.kind != LKS_OBJ_NONE && d->objective.mask) L.b_aux += L.F;
    if (d->rho_init || d->u_init) L.b_aux += nf * L.F * e;
    L.b_args = (size_t)N * (L.esz == 8 ? lks::args_bytes<double>() : lks::args_bytes<float>()) + 4096;
    L.bytes = L.b_state + L.b_ckpt + L.b_traj + L.b_box + L.b_kbar + L.b_adj + L.b_final +
              L.b_design + L.b_aux + L.b_pv + L.b_args + L.b_xring + L.b_padj;
    if (d->hbm_budget_bytes && L.bytes > d->hbm_budget_bytes)
        return fail(err, LKS_ENOMEM, "context needs " + std::to_string(L.bytes) +
                                          " bytes, over the HBM budget");
    return LKS_OK;
}

struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    int kind = 0;
};

}  // namespace

struct lks_ctx {
    lks_desc d{};
    Layout L;
    std::vector<lks_motion> motion;
    hipStream_t stream = nullptr;
    int dev = 0;
    // device memory
    char *state = nullptr, *ckpt = nullptr, *traj = nullptr, *box = nullptr, *kbar = nullptr,
         *adj = nullptr, *fin = nullptr, *gamma = nullptr, *kref = nullptr, *sens = nullptr,
         *kstatic = nullptr, *init = nullptr, *pv = nullptr, *xring = nullptr, *padj = nullptr;
    double *kprime = nullptr, *G = nullptr, *jn = nullptr, *partials = nullptr;
    unsigned int *counter = nullptr;
    int *flag = nullptr;
    uint8_t *mask = nullptr;
    std::vector<void *> allocs;
    double obj_scale = 0.0;
    bool have_fwd = false, have_adj = false;
    std::string err;
    // timing
    int every = 0;
    long launches[3] = {0, 0, 0};
    long samples[3] = {0, 0, 0};
    double total_ms[3] = {0, 0, 0};
    std::vector<EventPair> pool;
    size_t pool_used = 0;
    // continuous batching: where this context stands in its evaluation
    struct Cursor {
        int phase = 0;  // 0 idle, 1 forward, 2 reverse setup, 3 reverse (adjoint + recompute), 6 done
        int n = 0, seg = 0, cur = 0, acur = 0;
        int ready = 0, rseg = -1, rn = 0;  // reverse sweep: recompute of the previous segment
    } cs;
    double *jn_host = nullptr;  // pinned
    int *flag_host = nullptr;   // pinned
    // per-step kernel argument blocks of one sweep: built on the host, uploaded once per sweep
    char *argdev = nullptr;
    char *arghost = nullptr;    // pinned
    size_t argcap = 0;
    long long *tile0 = nullptr; // device {0}: the single job of a one-job launch
    void *out_dev = nullptr;    // caller's device buffer for dJ/dgamma
    hipEvent_t done_ev = nullptr;
    // reverse sweep: segments are recomputed on stream2 while the adjoint runs on stream
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_fork = nullptr, ev_rec = nullptr, ev_adj = nullptr;
    bool overlap = false;  // a recompute is in flight beside the adjoint launches (not timed)

    size_t esz() const { return L.esz; }
    int D() const { return d.dim; }
    char *field(char *base, long long slot_fields) const { return base + slot_fields * L.F * L.esz; }
};

namespace {

#define HIPCHK(ctx, expr)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) {                                                             \
            (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                 \
            return LKS_EDEVICE;                                                             \
        }                                                                                   \
    } while (0)

int dalloc(lks_ctx *c, size_t bytes, void **p) {
    if (bytes == 0) {
        *p = nullptr;
        return LKS_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        c->err = std::string("hipMalloc failed: ") + hipGetErrorString(e);
        *p = nullptr;
        return LKS_ENOMEM;
    }
    c->allocs.push_back(*p);
    return LKS_OK;
}

template <typename T>
lks::BCParams<T> bc_params(const lks_desc &d) {
    lks::BCParams<T> b{};
    for (int f = 0; f < 6; ++f) {
        b.kind[f] = (f / 2 < d.dim) ? d.bc[f].kind : LKS_BC_PERIODIC;
        b.rho[f] = (T)(d.bc[f].rho - 1.0);
        for (int a = 0; a < 3; ++a) b.u[f][a] = (a < d.dim) ? (T)d.bc[f].u[a] : T(0);
    }
    return b;
}

template <typename T>
lks::Design<T> design(const lks_ctx *c) {
    lks::Design<T> s{};
    s.kref = reinterpret_cast<const T *>(c->kref);
    for (int a = 0; a < 3; ++a) {
        s.nd[a] = c->d.nd[a];
        s.xiG[a] = a < c->d.dim ? c->d.xi_G[a] : 0.0;
    }
    s.weight = c->d.weight == LKS_W_LIN ? 1 : 0;
    return s;
}

lks::ObjParams obj_params(const lks_ctx *c, int n) {
    lks::ObjParams o{};
    const lks_objective &ob = c->d.objective;
    o.kind = ob.kind;
    o.active = ob.kind != LKS_OBJ_NONE && n >= ob.n0 && n <= ob.n1;
    o.scale = c->obj_scale;
    for (int a = 0; a < 3; ++a) {
        o.centre[a] = ob.centre[a];
        o.dir[a] = ob.dir[a];
    }
    o.mask = c->mask;
    o.partials = o.active ? c->partials + (long long)((n - ob.n0) % c->L.prow) * c->L.max_blocks : nullptr;
    return o;
}

// After forward step n: first step of the run of partial rows to reduce now (the ring is full or
// the window ends), or 0.
int reduce_from(const lks_ctx *c, int n) {
    const lks_objective &ob = c->d.objective;
    if (ob.kind == LKS_OBJ_NONE || n < ob.n0 || n > ob.n1) return 0;
    const int k = (n - ob.n0) % c->L.prow;
    return (k == c->L.prow - 1 || n == ob.n1) ? n - k : 0;
}

// ---- timing: sample every k-th launch of a kernel kind with an event pair ------------------
int flush_timing(lks_ctx *c) {
    if (c->pool_used == 0) return LKS_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->stream2) HIPCHK(c, hipStreamSynchronize(c->stream2));
    for (size_t i = 0; i < c->pool_used; ++i) {
        float ms = 0;
        HIPCHK(c, hipEventElapsedTime(&ms, c->pool[i].a, c->pool[i].b));
        c->samples[c->pool[i].kind] += 1;
        c->total_ms[c->pool[i].kind] += ms;
    }
    c->pool_used = 0;
    return LKS_OK;
}

struct Timed {
    lks_ctx *c;
    EventPair *ev = nullptr;
    hipStream_t s;
    // launches on the recompute stream overlap the adjoint stream, so their event pairs would
    // include queueing behind the other stream: only launches on the context's stream are timed
    Timed(lks_ctx *cc, int kind, hipStream_t st) : c(cc), s(st) {
        const long k = c->launches[kind]++;
        if (s == c->stream && !c->overlap && c->every > 0 && k % c->every == 0 &&
            c->pool_used < c->pool.size()) {
            ev = &c->pool[c->pool_used++];
            ev->kind = kind;
            (void)hipEventRecord(ev->a, s);
        }
    }
    ~Timed() {
        if (ev) (void)hipEventRecord(ev->b, s);
        if (ev && c->pool_used == c->pool.size()) (void)flush_timing(c);
    }
};

// Segment seg keeps its trajectory and footprint arrays in bank (S - 1 - seg) % 2: the last
// segment (written by the forward sweep) is in bank 0, and consecutive segments alternate, so
// segment seg - 1 can be recomputed while the adjoint of segment seg reads the other bank.
int bank_of(const lks_ctx *c, int seg) { return c->L.banks == 1 ? 0 : (c->L.S - 1 - seg) & 1; }

// kappa and u_S of one step on its footprint box: (1 + dim) arrays of box.cells values.  The
// forward sweep keeps them in a two-slot ring (step n in slot n % 2) except in the last segment,
// whose steps go to the box store (slot j - 1 for the j-th step of the segment) because the
// reverse sweep reads them; a recomputed segment writes the box store the same way.
template <typename T>
T *box_slot(lks_ctx *c, bool ring, int slot, int bank = 0) {
    const long long s = ring ? slot : (long long)bank * c->L.K + slot;
    return reinterpret_cast<T *>(ring ? c->xring : c->box) + s * (1 + c->d.dim) * c->L.box.cells;
}

template <typename T>
T *fwd_loc(lks_ctx *c, int n) {
    const int seg = (n - 1) / c->L.K;
    if (seg == c->L.S - 1 && !c->L.fwd_only)
        return box_slot<T>(c, false, n - seg * c->L.K - 1, bank_of(c, seg));
    return box_slot<T>(c, true, n & 1);
}

template <typename T>
T *rec_loc(lks_ctx *c, int seg, int n) {
    return box_slot<T>(c, false, n - seg * c->L.K - 1, bank_of(c, seg));
}

template <typename T>
lks::FwdArgs<T> base_fwd_args(lks_ctx *c) {
    lks::FwdArgs<T> a{};
    a.g = c->L.g;
    a.bc = bc_params<T>(c->d);
    a.A = (T)(4.5 * (1.0 / 6.0 - c->d.nu));
    for (int k = 0; k < 3; ++k) a.gf[k] = k < c->d.dim ? (T)c->d.body_force[k] : T(0);
    a.kstatic = reinterpret_cast<const T *>(c->kstatic);
    a.des = design<T>(c);
    a.box = c->L.box;
    return a;
}

template <typename T>
void set_next(lks_ctx *c, lks::FwdArgs<T> &a, int n, T *knext) {
    a.mode |= lks::FWD_TRANSFER_NEXT;
    if (c->d.weight == LKS_W_COS4) a.mode |= lks::FWD_TRANSFER_FIRST;
    a.mnext = c->L.steps[n];
    a.knext = knext;
    for (int k = 0; k < 3; ++k) a.usnext[k] = k < c->d.dim ? knext + (1 + k) * c->L.box.cells : nullptr;
}

// forward step n: reads kappa, u_S of step n at kin; if knext is set, its extra blocks transfer
// step n + 1 into knext
template <typename T>
lks::FwdArgs<T> make_fwd_args(lks_ctx *c, int n, const T *rin, const T *const uin[3], T *rout,
                              T *const uout[3], const T *kin, T *knext, bool objective) {
    lks::FwdArgs<T> a = base_fwd_args<T>(c);
    a.rin = rin;
    a.rout = rout;
    for (int k = 0; k < 3; ++k) {
        a.uin[k] = k < c->d.dim ? uin[k] : nullptr;
        a.uout[k] = k < c->d.dim ? uout[k] : nullptr;
    }
    a.m = c->L.steps[n];
    a.kin = kin;
    for (int k = 0; k < 3; ++k) a.usin[k] = k < c->d.dim ? kin + (1 + k) * c->L.box.cells : nullptr;
    a.mode = lks::FWD_STENCIL;
    if (knext) set_next<T>(c, a, n + 1, knext);
    a.obj = obj_params(c, n);
    if (!objective) a.obj.active = 0;
    return a;
}

// transfer-only launch: kappa, u_S of step n into kdst (before the first step of a sweep)
template <typename T>
lks::FwdArgs<T> make_xfer_args(lks_ctx *c, int n, T *kdst) {
    lks::FwdArgs<T> a = base_fwd_args<T>(c);
    a.m = c->L.steps[n];
    set_next<T>(c, a, n, kdst);
    return a;
}

// blocks of one forward launch: the stencil tiles, then the transfer blocks
long long fwd_tiles(const lks_ctx *c, int mode) {
    long long t = 0;
    if (mode & lks::FWD_STENCIL)
        t += c->d.dim == 2 ? lks::tiles2d_fwd(c->L.g) : lks::tiles3d(c->L.g, (int)c->L.esz);
    if (mode & lks::FWD_TRANSFER_NEXT) t += lks::xfer_blocks(c->d.dim, c->L.box.cells, (int)c->L.esz);
    return t;
}

// one-job launches: the argument block lives in device memory (see upload_args)
template <typename T>
hipError_t launch_fwd_raw(lks_ctx *c, const lks::FwdArgs<T> *dargs, long long ntiles, hipStream_t s) {
    return c->d.dim == 2 ? lks::launch_fwd2d_batch<T>(dargs, c->tile0, 1, ntiles, s)
                         : lks::launch_fwd3d_batch<T>(dargs, c->tile0, 1, ntiles, c->d.lattice, c->L.g.per[2] != 0, s);
}

// one forward step (timed as kind 0); mode is the host copy's mode
template <typename T>
int launch_fwd_dev(lks_ctx *c, const lks::FwdArgs<T> *dargs, int mode, hipStream_t s) {
    hipError_t e;
    {
        Timed t(c, 0, s);
        e = launch_fwd_raw<T>(c, dargs, fwd_tiles(c, mode), s);
    }
    HIPCHK(c, e);
    return LKS_OK;
}

// transfer-only launch (not part of the per-step timing); in 3D a kernel without LDS
template <typename T>
int launch_xfer_dev(lks_ctx *c, const lks::FwdArgs<T> *dargs, hipStream_t s) {
    if (c->d.dim == 3)
        HIPCHK(c, (lks::launch_xfer3d_batch<T>(dargs, c->tile0, 1, fwd_tiles(c, lks::FWD_TRANSFER_NEXT), s)));
    else
        HIPCHK(c, (launch_fwd_raw<T>(c, dargs, fwd_tiles(c, lks::FWD_TRANSFER_NEXT), s)));
    return LKS_OK;
}

// one recomputed 3D step of the reverse sweep: the stencil tiles (with their LDS), then the
// transfer of the next step as a launch of its own without LDS.  Fused, the transfer's many
// short blocks each held the stencil's LDS and kept the adjoint launches of the other stream
// waiting for it.
template <typename T>
int launch_fwd_split3(lks_ctx *c, const lks::FwdArgs<T> *dargs, int mode, hipStream_t s) {
    hipError_t e;
    {
        Timed t(c, 0, s);
        e = launch_fwd_raw<T>(c, dargs, fwd_tiles(c, mode & lks::FWD_STENCIL), s);
        if (e == hipSuccess && (mode & lks::FWD_TRANSFER_NEXT))
            e = lks::launch_xfer3d_batch<T>(dargs, c->tile0, 1, fwd_tiles(c, lks::FWD_TRANSFER_NEXT), s);
    }
    HIPCHK(c, e);
    return LKS_OK;
}

// one adjoint step; in 2D its launch also carries the gather of the previous adjoint step
// (extra blocks, host copy `ha` says how many)
template <typename T>
int launch_adj_fused(lks_ctx *c, const lks::AdjArgs<T> *dargs, const lks::AdjArgs<T> &ha) {
    hipError_t e;
    {
        Timed t(c, 1, c->stream);
        e = lks::launch_adj2d_batch<T>(dargs, c->tile0, 1,
                                       lks::tiles2d(c->L.g) + (ha.sens ? ha.sens_blocks : 0), c->stream);
    }
    HIPCHK(c, e);
    return LKS_OK;
}

template <typename T>
int launch_sens_dev(lks_ctx *c, const lks::SensArgs<T> *dsens) {
    hipError_t e;
    {
        Timed t(c, 2, c->stream);
        e = lks::launch_sens_batch<T>(dsens, c->tile0, 1, (c->L.nd + lks::kBlockHost - 1) / lks::kBlockHost,
                                      c->stream);
    }
    HIPCHK(c, e);
    return LKS_OK;
}

template <typename T>
int launch_adj_dev(lks_ctx *c, const lks::AdjArgs<T> *dargs, const lks::SensArgs<T> *dsens) {
    hipError_t e;
    {
        Timed t(c, 1, c->stream);
        e = c->d.dim == 2
                ? lks::launch_adj2d_batch<T>(dargs, c->tile0, 1, lks::tiles2d(c->L.g), c->stream)
                : lks::launch_adj3d_batch<T>(dargs, c->tile0, lks::prep_blocks3(c->L.ncell),
                                             c->tile0, lks::tiles3d_adj(c->L.g, (int)c->L.esz), 1,
                                             c->d.lattice, c->L.g.per[2] != 0, c->stream);
    }
    HIPCHK(c, e);
    {
        Timed t(c, 2, c->stream);
        e = lks::launch_sens_batch<T>(dsens, c->tile0, 1, (c->L.nd + lks::kBlockHost - 1) / lks::kBlockHost,
                                      c->stream);
    }
    HIPCHK(c, e);
    return LKS_OK;
}

// copy `bytes` of argument blocks (already written to the pinned staging area) to the device
int upload_args(lks_ctx *c, size_t bytes) {
    if (bytes > c->argcap) {
        c->err = "argument staging area too small";
        return LKS_EINVAL;
    }
    HIPCHK(c, hipMemcpyAsync(c->argdev, c->arghost, bytes, hipMemcpyHostToDevice, c->stream));
    return LKS_OK;
}

template <typename T>
struct Fields {
    T *r;
    T *u[3];
};

template <typename T>
Fields<T> state_fields(lks_ctx *c, char *base) {  // (1 + dim) consecutive fields
    Fields<T> f{};
    f.r = reinterpret_cast<T *>(base);
    for (int k = 0; k < 3; ++k)
        f.u[k] = k < c->d.dim ? reinterpret_cast<T *>(c->field(base, 1 + k)) : nullptr;
    return f;
}

template <typename T>
void traj_slot(lks_ctx *c, int bank, int j, T *u[3]) {  // dim consecutive fields per slot
    const long long slot = (long long)bank * (c->L.K + 1) + j;
    for (int k = 0; k < 3; ++k)
        u[k] = k < c->d.dim ? reinterpret_cast<T *>(c->field(c->traj, slot * c->d.dim + k)) : nullptr;
}

template <typename T>
int copy_fields(lks_ctx *c, T *dst, const T *src, int nfields, hipStream_t s = nullptr) {
    HIPCHK(c, hipMemcpyAsync(dst, src, (size_t)nfields * c->L.F * sizeof(T), hipMemcpyDeviceToDevice,
                             s ? s : c->stream));
    return LKS_OK;
}

// Non-finite guard: flag[0] = first forward step whose state held a NaN/Inf (INT_MAX: none),
// flag[1] = largest n whose reverse step produced a non-finite adjoint state (0: none), flag[2] = 1
// if G held a NaN/Inf.  Filled by kernels (no memset node), so the sequence stays capturable.
int reset_flags(lks_ctx *c, bool fwd, hipStream_t s) {
    if (fwd) HIPCHK(c, lks::launch_fill<int>(c->flag, INT_MAX, 1, s));
    HIPCHK(c, lks::launch_fill<int>(c->flag + 1, 0, 2, s));
    return LKS_OK;
}

bool scan_fwd_step(const lks_ctx *c, int n) { return n % lks::kScanEvery == 0 || n == c->d.nsteps; }
bool scan_adj_step(int n) { return (n - 1) % lks::kScanEvery == 0; }

// scan the state a forward step wrote (rho - 1 and the dim velocity fields, each run contiguous)
template <typename T>
int scan_fwd(lks_ctx *c, const lks::FwdArgs<T> &a, int n, hipStream_t s) {
    HIPCHK(c, lks::launch_scan<T>(a.rout, c->L.F, a.uout[0], (long long)c->d.dim * c->L.F, n, c->flag, 0, s));
    return LKS_OK;
}

template <typename T>
int scan_adj(lks_ctx *c, const lks::AdjArgs<T> &a, int n, hipStream_t s) {
    HIPCHK(c, lks::launch_scan<T>(a.Pout, c->L.F, a.Vout[0], (long long)c->d.dim * c->L.F, n, c->flag + 1, 1, s));
    return LKS_OK;
}

int nonfinite_error(lks_ctx *c, const int f[3]) {
    char buf[256];
    if (f[0] != INT_MAX) {
        const int prev = f[0] == c->d.nsteps && f[0] % lks::kScanEvery ? f[0] - f[0] % lks::kScanEvery
                                                                       : f[0] - lks::kScanEvery;
        std::snprintf(buf, sizeof buf,
                      "non-finite forward state first seen after step %d (scanned every %d steps; finite "
                      "after step %d)", f[0], lks::kScanEvery, prev > 0 ? prev : 0);
    } else if (f[1] != 0) {
        std::snprintf(buf, sizeof buf,
                      "non-finite adjoint state first seen after the reverse step of n = %d (scanned every "
                      "%d steps)", f[1], lks::kScanEvery);
    } else if (f[2] != 0) {
        std::snprintf(buf, sizeof buf, "non-finite value in the design sensitivity G");
    } else {
        return LKS_OK;
    }
    c->err = buf;
    return LKS_ENONFINITE;
}

template <typename T>
int forward_impl(lks_ctx *c, const void *gamma, double *J) {
    const Layout &L = c->L;
    const int D = c->d.dim, N = c->d.nsteps, K = L.K, S = L.S;
    int rc;
    c->have_fwd = c->have_adj = false;
    HIPCHK(c, hipMemcpyAsync(c->gamma, gamma, L.nd * sizeof(T), hipMemcpyDefault, c->stream));
    HIPCHK(c, lks::launch_design_prep<T>(reinterpret_cast<const T *>(c->gamma),
                                         reinterpret_cast<T *>(c->kref), c->kprime, L.nd,
                                         c->d.interp == LKS_INTERP_PAPER ? 0 : 1,
                                         c->d.kappa_max, c->d.q, c->stream));
    HIPCHK(c, lks::launch_fill<double>(c->jn, 0.0, N + 1, c->stream));
    if ((rc = reset_flags(c, true, c->stream))) return rc;

    Fields<T> st[2] = {state_fields<T>(c, c->state), state_fields<T>(c, c->field(c->state, 1 + D))};
    {
        lks::InitArgs<T> ia{};
        ia.g = L.g;
        ia.bc = bc_params<T>(c->d);
        ia.r0 = (T)(c->d.rho0 - 1.0);
        for (int k = 0; k < 3; ++k) ia.u0[k] = k < D ? (T)c->d.u0[k] : T(0);
        if (c->init) {
            Fields<T> in = state_fields<T>(c, c->init);
            ia.rinit = in.r;
            for (int k = 0; k < 3; ++k) ia.uinit[k] = in.u[k];
        }
        ia.rout = st[0].r;
        for (int k = 0; k < 3; ++k) ia.uout[k] = st[0].u[k];
        HIPCHK(c, lks::launch_init<T>(ia, c->stream));
    }
    // argument blocks of every step of the sweep (the pointer pattern is fixed in advance)
    {
        auto *fa = reinterpret_cast<lks::FwdArgs<T> *>(c->arghost);
        int cur = 0;
        for (int n = 1; n <= N; ++n) {
            const int seg = (n - 1) / K, j = n - seg * K;
            const bool last = seg == S - 1 && !L.fwd_only;
            T *uin[3], *uout[3];
            if (last) {
                traj_slot<T>(c, 0, j - 1, uin);
                traj_slot<T>(c, 0, j, uout);
            } else {
                for (int k = 0; k < 3; ++k) {
                    uin[k] = st[cur].u[k];
                    uout[k] = st[1 - cur].u[k];
                }
            }
            fa[n - 1] = make_fwd_args<T>(c, n, st[cur].r, uin, st[1 - cur].r, uout, fwd_loc<T>(c, n),
                                         n < N ? fwd_loc<T>(c, n + 1) : nullptr, true);
            cur = 1 - cur;
        }
        fa[N] = make_xfer_args<T>(c, 1, fwd_loc<T>(c, 1));
        if (D == 2)
            for (int n = 1; n < N; ++n)  // the launch of step n prefetches that of step n + 1
                fa[n - 1].next = reinterpret_cast<const lks::FwdArgs<T> *>(c->argdev) + n;
        if ((rc = upload_args(c, (size_t)(N + 1) * sizeof(lks::FwdArgs<T>)))) return rc;
    }
    const auto *dfa = reinterpret_cast<const lks::FwdArgs<T> *>(c->argdev);
    const auto *hfa = reinterpret_cast<const lks::FwdArgs<T> *>(c->arghost);
    if ((rc = launch_xfer_dev<T>(c, dfa + N, c->stream))) return rc;
    int cur = 0;
    for (int n = 1; n <= N; ++n) {
        const int seg = (n - 1) / K, j = n - seg * K;
        const bool last = seg == S - 1 && !L.fwd_only;
        if (j == 1) {
            T *ck = reinterpret_cast<T *>(c->field(c->ckpt, (long long)seg * (1 + D)));
            if ((rc = copy_fields<T>(c, ck, st[cur].r, 1))) return rc;
            if ((rc = copy_fields<T>(c, reinterpret_cast<T *>(c->field(reinterpret_cast<char *>(ck), 1)),
                                     st[cur].u[0], D)))
                return rc;
            if (last) {
                T *t0[3];
                traj_slot<T>(c, 0, 0, t0);
                if ((rc = copy_fields<T>(c, t0[0], st[cur].u[0], D))) return rc;
            }
        }
        if ((rc = launch_fwd_dev<T>(c, dfa + (n - 1), hfa[n - 1].mode, c->stream))) return rc;
        if (scan_fwd_step(c, n) && (rc = scan_fwd<T>(c, hfa[n - 1], n, c->stream))) return rc;
        if (const int na = reduce_from(c, n))  // j^na .. j^n, each in block order
            HIPCHK(c, lks::launch_reduce_steps(c->partials, L.max_blocks, L.max_blocks, na, n, c->obj_scale,
                                               c->jn, c->stream));
        cur = 1 - cur;
    }
    // keep X^N: the trajectory store is reused by the reverse sweep
    {
        Fields<T> fin = state_fields<T>(c, c->fin);
        T *ul[3];
        if (L.fwd_only) {
            for (int k = 0; k < 3; ++k) ul[k] = st[cur].u[k];
        } else {
            traj_slot<T>(c, 0, N - (S - 1) * K, ul);
        }
        if ((rc = copy_fields<T>(c, fin.r, st[cur].r, 1))) return rc;
        if ((rc = copy_fields<T>(c, fin.u[0], ul[0], D))) return rc;
    }
    std::vector<double> jn(N + 1);
    int flag[3] = {0, 0, 0};
    HIPCHK(c, hipMemcpyAsync(jn.data(), c->jn, (N + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(flag, c->flag, sizeof flag, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((rc = flush_timing(c))) return rc;
    double acc = 0.0;
    for (int n = 0; n <= N; ++n) acc += jn[n];
    if (J) *J = acc;
    if ((rc = nonfinite_error(c, flag))) return rc;
    c->have_fwd = true;
    return LKS_OK;
}

template <typename T>
lks::AdjArgs<T> make_adj_args(lks_ctx *c, int n, int j, int acur) {
    const Layout &L = c->L;
    const int D = c->d.dim;
    Fields<T> ad[2] = {state_fields<T>(c, c->adj), state_fields<T>(c, c->field(c->adj, 1 + D))};
    lks::AdjArgs<T> a{};
    a.g = L.g;
    a.bc = bc_params<T>(c->d);
    a.A = (T)(4.5 * (1.0 / 6.0 - c->d.nu));
    a.Pin = ad[acur].r;
    a.Pout = ad[1 - acur].r;
    T *up[3], *uc[3];
    const int bank = bank_of(c, (n - 1) / L.K);
    traj_slot<T>(c, bank, j - 1, up);
    traj_slot<T>(c, bank, j, uc);
    for (int k = 0; k < 3; ++k) {
        a.Vin[k] = ad[acur].u[k];
        a.Vout[k] = ad[1 - acur].u[k];
        a.uprev[k] = up[k];
        a.ucur[k] = uc[k];
    }
    a.kstatic = reinterpret_cast<const T *>(c->kstatic);
    const T *b = box_slot<T>(c, false, j - 1, bank);
    a.kbox = b;
    for (int k = 0; k < 3; ++k) a.usbox[k] = k < D ? b + (1 + k) * L.box.cells : nullptr;
    a.kbar = reinterpret_cast<T *>(c->kbar) + (long long)(n & 1) * L.box.cells;
    a.box = L.box;
    a.m = L.steps[n];
    a.obj = obj_params(c, n);
    if (c->pv) {
        a.Ps = reinterpret_cast<T *>(c->pv);
        for (int k = 0; k < 3; ++k) a.Vs[k] = reinterpret_cast<T *>(c->field(c->pv, 1 + k));
    }
    return a;
}

// the paper's adjoint form: (P*, V*) scratch, 3 u~ ping-pong (in slot acur, out slot 1 - acur), s~
template <typename T>
void set_paper_args(lks_ctx *c, lks::AdjArgs<T> &a, int acur) {
    const int D = c->d.dim;
    T *b = reinterpret_cast<T *>(c->padj);
    const long long F = c->L.F;
    a.Ps = b;
    for (int k = 0; k < 3; ++k) {
        a.Vs[k] = k < D ? b + (1 + k) * F : nullptr;
        a.U3in[k] = k < D ? b + (1 + D + acur * D + k) * F : nullptr;
        a.U3out[k] = k < D ? b + (1 + D + (1 - acur) * D + k) * F : nullptr;
        a.st[k] = b + (1 + 3 * D + k) * F;
    }
}

template <typename T>
lks::SensArgs<T> make_sens_args(lks_ctx *c, int n) {
    lks::SensArgs<T> sa{};
    sa.kbar = reinterpret_cast<T *>(c->kbar) + (long long)(n & 1) * c->L.box.cells;
    sa.box = c->L.box;
    sa.m = c->L.steps[n];
    sa.des = design<T>(c);
    sa.dim = c->d.dim;
    sa.G = c->G;
    return sa;
}

// Reverse sweep, segments last to first.  The adjoint of segment seg runs on the context's
// stream while segment seg - 1 is restored from its checkpoint and recomputed on stream2 into
// the other trajectory/footprint bank: the two launch sequences are independent and each is
// latency-bound, so they share the GPU.  Events order the banks: the recompute of seg - 1 waits
// for the adjoint of seg + 1 (same bank), the adjoint of seg waits for its recompute.
template <typename T>
int adjoint_impl(lks_ctx *c) {
    const Layout &L = c->L;
    const int D = c->d.dim, N = c->d.nsteps, K = L.K, S = L.S;
    int rc;
    Fields<T> st[2] = {state_fields<T>(c, c->state), state_fields<T>(c, c->field(c->state, 1 + D))};
    Fields<T> ad = state_fields<T>(c, c->adj);
    // argument blocks: recomputed steps (every segment but the last), one transfer-only block per
    // recomputed segment, then the adjoint steps and the gathers
    const int nrec = (S - 1) * K, nfa = nrec + (S - 1);
    const bool paper = c->d.adjoint_form == LKS_ADJ_PAPER;
    auto *ra = reinterpret_cast<lks::FwdArgs<T> *>(c->arghost);
    auto *aa = reinterpret_cast<lks::AdjArgs<T> *>(c->arghost + (size_t)nfa * sizeof(lks::FwdArgs<T>));
    auto *sa = reinterpret_cast<lks::SensArgs<T> *>(reinterpret_cast<char *>(aa) + (size_t)N * sizeof(lks::AdjArgs<T>));
    const size_t bytes = (size_t)nfa * sizeof(lks::FwdArgs<T>) + (size_t)N * (sizeof(lks::AdjArgs<T>) + sizeof(lks::SensArgs<T>));
    {
        int acur = 0;
        for (int seg = S - 1; seg >= 0; --seg) {
            const int n0 = seg * K + 1, n1 = std::min((seg + 1) * K, N);
            if (seg != S - 1) {
                const int bank = bank_of(c, seg);
                int cur = 0;
                for (int n = n0; n <= n1; ++n) {
                    const int j = n - seg * K;
                    T *uin[3], *uout[3];
                    traj_slot<T>(c, bank, j - 1, uin);
                    traj_slot<T>(c, bank, j, uout);
                    ra[n - 1] = make_fwd_args<T>(c, n, st[cur].r, uin, st[1 - cur].r, uout, rec_loc<T>(c, seg, n),
                                                 n < n1 ? rec_loc<T>(c, seg, n + 1) : nullptr, false);
                    cur = 1 - cur;
                }
                ra[nrec + seg] = make_xfer_args<T>(c, n0, rec_loc<T>(c, seg, n0));
                if (D == 2)
                    for (int n = n0; n < n1; ++n)  // recomputed step n prefetches step n + 1
                        ra[n - 1].next = reinterpret_cast<const lks::FwdArgs<T> *>(c->argdev) + n;
            }
            for (int n = n1; n >= n0; --n) {
                aa[n - 1] = make_adj_args<T>(c, n, n - seg * K, acur);
                if (paper) set_paper_args<T>(c, aa[n - 1], acur);
                sa[n - 1] = make_sens_args<T>(c, n);
                acur = 1 - acur;
            }
        }
        if (D == 2 && !paper)  // the adjoint launch of step n prefetches that of step n - 1
            for (int n = 2; n <= N; ++n)
                aa[n - 1].next = reinterpret_cast<const lks::AdjArgs<T> *>(c->argdev + (size_t)nfa * sizeof(lks::FwdArgs<T>)) + (n - 2);
        if (D == 2 && !paper) {  // each adjoint launch also runs the gather of the step after it (kappa_bar
                       // of consecutive steps lives in alternate halves of the kappa_bar buffer)
            const auto *dsa_dev = reinterpret_cast<const lks::SensArgs<T> *>(
                c->argdev + (size_t)nfa * sizeof(lks::FwdArgs<T>) + (size_t)N * sizeof(lks::AdjArgs<T>));
            const long long sb = (L.nd + lks::kBlockHost - 1) / lks::kBlockHost;
            for (int n = 1; n < N; ++n) {
                aa[n - 1].sens = dsa_dev + n;
                aa[n - 1].sens_blocks = sb;
            }
        }
        if ((rc = upload_args(c, bytes))) return rc;
    }
    const auto *dra = reinterpret_cast<const lks::FwdArgs<T> *>(c->argdev);
    const auto *daa = reinterpret_cast<const lks::AdjArgs<T> *>(c->argdev + (size_t)nfa * sizeof(lks::FwdArgs<T>));
    const auto *dsa = reinterpret_cast<const lks::SensArgs<T> *>(reinterpret_cast<const char *>(daa) + (size_t)N * sizeof(lks::AdjArgs<T>));
    HIPCHK(c, lks::launch_fill<T>(ad.r, T(0), (long long)(1 + D) * L.F, c->stream));
    if (paper)  // 3 u~ of level N starts at zero like lambda^N
        HIPCHK(c, lks::launch_fill<T>(reinterpret_cast<T *>(c->padj), T(0), (long long)(1 + 3 * D) * L.F, c->stream));
    HIPCHK(c, lks::launch_fill<double>(c->G, 0.0, L.nd, c->stream));
    if ((rc = reset_flags(c, false, c->stream))) return rc;
    hipStream_t sr = c->stream2 ? c->stream2 : c->stream;  // recompute stream
    if (S > 1 && c->stream2) {  // stream2 starts after everything enqueued so far
        HIPCHK(c, hipEventRecord(c->ev_fork, c->stream));
        HIPCHK(c, hipStreamWaitEvent(c->stream2, c->ev_fork, 0));
    }
    for (int seg = S - 1; seg >= 0; --seg) {
        const int n0 = seg * K + 1, n1 = std::min((seg + 1) * K, N);
        if (seg != S - 1 && sr != c->stream)  // segment seg was recomputed on stream2
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->ev_rec, 0));
        if (seg >= 1) {  // restore and recompute segment seg - 1 into the other bank
            const int ps = seg - 1, p0 = ps * K + 1, p1 = std::min((ps + 1) * K, N);
            if (seg != S - 1 && sr != c->stream) HIPCHK(c, hipStreamWaitEvent(sr, c->ev_adj, 0));
            const T *ck = reinterpret_cast<const T *>(c->field(c->ckpt, (long long)ps * (1 + D)));
            T *t0[3];
            traj_slot<T>(c, bank_of(c, ps), 0, t0);
            if ((rc = copy_fields<T>(c, st[0].r, ck, 1, sr))) return rc;
            if ((rc = copy_fields<T>(c, t0[0], ck + L.F, D, sr))) return rc;
            if ((rc = launch_xfer_dev<T>(c, dra + nrec + ps, sr))) return rc;
            for (int n = p0; n <= p1; ++n)
                if ((rc = D == 3 ? launch_fwd_split3<T>(c, dra + (n - 1), ra[n - 1].mode, sr)
                                 : launch_fwd_dev<T>(c, dra + (n - 1), ra[n - 1].mode, sr)))
                    return rc;
            if (sr != c->stream) HIPCHK(c, hipEventRecord(c->ev_rec, sr));
        }
        c->overlap = seg >= 1 && sr != c->stream;
        for (int n = n1; n >= n0; --n) {
            if (paper) {
                {
                    Timed t(c, 1, c->stream);
                    HIPCHK(c, lks::launch_padj2d<T>(daa + (n - 1), L.g, c->stream));
                }
                rc = launch_sens_dev<T>(c, dsa + (n - 1));
            } else if (D == 2) {
                rc = launch_adj_fused<T>(c, daa + (n - 1), aa[n - 1]);
            } else {
                rc = launch_adj_dev<T>(c, daa + (n - 1), dsa + (n - 1));
            }
            if (rc) return rc;
            if (scan_adj_step(n) && (rc = scan_adj<T>(c, aa[n - 1], n, c->stream))) return rc;
        }
        c->overlap = false;
        if (sr != c->stream) HIPCHK(c, hipEventRecord(c->ev_adj, c->stream));
    }
    if (D == 2 && !paper && (rc = launch_sens_dev<T>(c, dsa))) return rc;  // gather of step 1
    HIPCHK(c, lks::launch_scan<double>(c->G, L.nd, nullptr, 0, 1, c->flag + 2, 1, c->stream));
    int flag[3] = {INT_MAX, 0, 0};
    HIPCHK(c, hipMemcpyAsync(flag + 1, c->flag + 1, 2 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (sr != c->stream) HIPCHK(c, hipStreamSynchronize(sr));
    if ((rc = flush_timing(c))) return rc;
    if ((rc = nonfinite_error(c, flag))) return rc;
    c->have_adj = true;
    return LKS_OK;
}

template <typename T>
int upload_padded(lks_ctx *c, char *dst, const double *src, int nfields) {
    const Layout &L = c->L;
    std::vector<T> h((size_t)nfields * L.F, T(0));
    for (int f = 0; f < nfields; ++f)
        for (long long z = 0; z < L.g.n[2]; ++z)
            for (long long y = 0; y < L.g.n[1]; ++y)
                for (long long x = 0; x < L.g.n[0]; ++x)
                    h[f * L.F + x + y * L.g.sy + z * L.g.sz] =
                        (T)src[f * L.ncell + x + L.g.n[0] * (y + L.g.n[1] * z)];
    HIPCHK(c, hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return LKS_OK;
}

int create_impl(const lks_desc *d, lks_ctx *c) {
    int rc;
    c->d = *d;
    c->motion.assign(d->motion, d->motion + d->nsteps + 1);
    c->d.motion = c->motion.data();
    c->stream = reinterpret_cast<hipStream_t>(d->stream);
    HIPCHK(c, hipGetDevice(&c->dev));
    const Layout &L = c->L;
    const int D = d->dim;
    const size_t e = L.esz;
    void *p;
#define ALLOC(member, bytes)                                        \
    if ((rc = dalloc(c, (bytes), &p)) != LKS_OK) return rc;         \
    c->member = reinterpret_cast<decltype(c->member)>(p);
    ALLOC(state, L.b_state)
    ALLOC(ckpt, L.b_ckpt)
    ALLOC(traj, L.b_traj)
    ALLOC(box, L.b_box)
    ALLOC(xring, L.b_xring)
    ALLOC(kbar, L.b_kbar)
    ALLOC(adj, L.b_adj)
    ALLOC(fin, L.b_final)
    ALLOC(pv, L.b_pv)
    ALLOC(padj, L.b_padj)
    ALLOC(argdev, L.b_args)
    c->argcap = L.b_args - 256;  // the last 256 bytes hold tile0
    if (hipHostMalloc(reinterpret_cast<void **>(&c->arghost), L.b_args, 0) != hipSuccess) {
        c->arghost = nullptr;
        c->err = "pinned host allocation failed";
        return LKS_ENOMEM;
    }
    c->tile0 = reinterpret_cast<long long *>(c->argdev + L.b_args - 256);
    ALLOC(gamma, L.nd * e)
    ALLOC(kref, L.nd * e)
    ALLOC(sens, L.nd * e)
    ALLOC(kprime, L.nd * 8)
    ALLOC(G, L.nd * 8)
    ALLOC(jn, (d->nsteps + 1) * 8)
    ALLOC(partials, (size_t)L.prow * L.max_blocks * 8)
    ALLOC(counter, 64)
    if (L.banks == 2) {  // recompute stream for the reverse sweep (default priority)
        HIPCHK(c, hipStreamCreateWithFlags(&c->stream2, hipStreamNonBlocking));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_rec, hipEventDisableTiming));
        HIPCHK(c, hipEventCreateWithFlags(&c->ev_adj, hipEventDisableTiming));
    }
    c->flag = reinterpret_cast<int *>(reinterpret_cast<char *>(c->counter) + 32);
    HIPCHK(c, hipMemset(c->counter, 0, 64));
    HIPCHK(c, hipMemset(c->tile0, 0, 256));
    // padded row tails are never written by the kernels: start every field buffer at zero
    for (char *b : {c->state, c->ckpt, c->traj, c->adj, c->fin, c->padj})
        if (b) HIPCHK(c, hipMemset(b, 0, b == c->state ? L.b_state : b == c->ckpt ? L.b_ckpt
                                         : b == c->traj ? L.b_traj : b == c->adj ? L.b_adj
                                         : b == c->padj ? L.b_padj : L.b_final));
    if (d->kappa_static) {
        ALLOC(kstatic, L.F * e)
        rc = e == 8 ? upload_padded<double>(c, c->kstatic, d->kappa_static, 1)
                    : upload_padded<float>(c, c->kstatic, d->kappa_static, 1);
        if (rc) return rc;
    }
    if (d->rho_init || d->u_init) {
        ALLOC(init, (1 + D) * L.F * e)
        std::vector<double> h((size_t)(1 + D) * L.ncell);
        for (long long i = 0; i < L.ncell; ++i) h[i] = (d->rho_init ? d->rho_init[i] : d->rho0) - 1.0;
        for (int k = 0; k < D; ++k)
            for (long long i = 0; i < L.ncell; ++i)
                h[(1 + k) * L.ncell + i] = d->u_init ? d->u_init[k * L.ncell + i] : d->u0[k];
        rc = e == 8 ? upload_padded<double>(c, c->init, h.data(), 1 + D)
                    : upload_padded<float>(c, c->init, h.data(), 1 + D);
        if (rc) return rc;
    }
    long long mcount = L.ncell;
    if (d->objective.kind != LKS_OBJ_NONE && d->objective.mask) {
        ALLOC(mask, L.F)
        std::vector<uint8_t> h(L.F, 0);
        mcount = 0;
        for (long long z = 0; z < L.g.n[2]; ++z)
            for (long long y = 0; y < L.g.n[1]; ++y)
                for (long long x = 0; x < L.g.n[0]; ++x) {
                    const uint8_t v = d->objective.mask[x + L.g.n[0] * (y + L.g.n[1] * z)] ? 1 : 0;
                    h[x + y * L.g.sy + z * L.g.sz] = v;
                    mcount += v;
                }
        HIPCHK(c, hipMemcpy(c->mask, h.data(), L.F, hipMemcpyHostToDevice));
    }
#undef ALLOC
    c->d.rho_init = c->d.u_init = c->d.kappa_static = nullptr;
    c->d.objective.mask = nullptr;
    c->obj_scale = 1.0;
    if (d->objective.normalize & LKS_NORM_TIME) c->obj_scale /= (double)(d->objective.n1 - d->objective.n0 + 1);
    if (d->objective.normalize & LKS_NORM_MASK) c->obj_scale /= (double)std::max(1LL, mcount);
    return LKS_OK;
}

// ---- forward sweep without device allocation -------------------------------------------------
// Every buffer the forward kernels use beyond the caller's gamma and outputs is carved out of one
// static device array (`scratch`).  In host code the array's name is only a stand-in for the
// symbol: its device address is taken with hipGetSymbolAddress once per device, with that device
// current, and only that address is ever handed to kernels or copies.
constexpr size_t kScratchBytes = LKS_NOALLOC_SCRATCH_BYTES;

}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's copy of `scratch` (set up on the first call on the device)
int scratch_address(void **out, std::string *err) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(err, LKS_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(err, LKS_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(err, LKS_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return LKS_OK;
}

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

template <typename T>
int forward_noalloc_impl(const lks_desc *d, const void *gamma, double *J, void *drho, void *u,
                         std::string *err) {
    lks_ctx c;  // host bookkeeping only: its device pointers all point into the scratch
    int rc = plan(d, c.L, err);
    if (rc) return rc;
    Layout &L = c.L;
    const int D = d->dim, N = d->nsteps;
    // the forward sweep alone: X^0 is the only checkpoint and no trajectory is stored
    L.fwd_only = true;
    L.K = N;
    L.S = 1;
    L.banks = 1;
    const size_t e = L.esz, nf = 1 + D, fb = (size_t)L.F * e;
    const bool has_mask = d->objective.kind != LKS_OBJ_NONE && d->objective.mask;
    struct Part {
        char **dst;
        size_t bytes;
    };
    char *argdev = nullptr, *counter = nullptr, *kprime = nullptr, *jn = nullptr, *partials = nullptr;
    const size_t args_bytes = (size_t)(N + 1) * sizeof(lks::FwdArgs<T>);
    const Part parts[] = {
        {&c.state, 2 * nf * fb},
        {&c.ckpt, nf * fb},
        {&c.fin, nf * fb},
        {&c.xring, L.b_xring},
        {&c.gamma, (size_t)L.nd * e},
        {&c.kref, (size_t)L.nd * e},
        {&kprime, (size_t)L.nd * 8},
        {&jn, (size_t)(N + 1) * 8},
        {&partials, (size_t)L.prow * L.max_blocks * 8},
        {&counter, 64},
        {&c.kstatic, d->kappa_static ? fb : 0},
        {reinterpret_cast<char **>(&c.mask), has_mask ? (size_t)L.F : 0},
        {&c.init, (d->rho_init || d->u_init) ? nf * fb : 0},
        {&argdev, args_bytes + 256},  // + tile0
    };
    size_t need = 0;
    for (const Part &pt : parts) need += align256(pt.bytes);
    if (need > kScratchBytes)
        return fail(err, LKS_EINVAL,
                    "this forward sweep needs " + std::to_string(need) + " bytes of scratch; the static scratch "
                    "holds " + std::to_string(kScratchBytes) + " (use lks_create / lks_forward)");
    void *base = nullptr;
    if ((rc = scratch_address(&base, err))) return rc;
    size_t off = 0;
    for (const Part &pt : parts) {
        *pt.dst = pt.bytes ? static_cast<char *>(base) + off : nullptr;
        off += align256(pt.bytes);
    }
    c.kprime = reinterpret_cast<double *>(kprime);
    c.jn = reinterpret_cast<double *>(jn);
    c.partials = reinterpret_cast<double *>(partials);
    c.counter = reinterpret_cast<unsigned int *>(counter);
    c.flag = reinterpret_cast<int *>(counter + 32);
    c.argdev = argdev;
    c.argcap = args_bytes;
    c.tile0 = reinterpret_cast<long long *>(argdev + args_bytes);
    std::vector<char> staging(args_bytes);  // host staging of the argument blocks
    c.arghost = staging.data();
    c.d = *d;
    c.d.motion = nullptr;  // the plan holds every step's motion
    c.stream = reinterpret_cast<hipStream_t>(d->stream);
    hipError_t he = hipGetDevice(&c.dev);
    if (he != hipSuccess) return fail(err, LKS_EDEVICE, hipGetErrorString(he));
    // the scratch keeps the previous call's contents: clear what must start at zero (the padded
    // row tails of the fields, which the kernels never write, the counters and the job table)
    rc = LKS_OK;
    auto check = [&](hipError_t x) {
        if (x != hipSuccess && rc == LKS_OK) rc = fail(err, LKS_EDEVICE, hipGetErrorString(x));
    };
    check(lks::launch_fill<T>(reinterpret_cast<T *>(c.state), T(0), (long long)(2 * nf * L.F), c.stream));
    check(lks::launch_fill<int>(reinterpret_cast<int *>(counter), 0, 16, c.stream));
    check(lks::launch_fill<int>(reinterpret_cast<int *>(c.tile0), 0, 64, c.stream));
    if (rc) return rc;
    if (d->kappa_static) {
        rc = upload_padded<T>(&c, c.kstatic, d->kappa_static, 1);
        if (rc) return fail(err, rc, c.err);
    }
    if (d->rho_init || d->u_init) {
        std::vector<double> h(nf * (size_t)L.ncell);
        for (long long i = 0; i < L.ncell; ++i) h[i] = (d->rho_init ? d->rho_init[i] : d->rho0) - 1.0;
        for (int k = 0; k < D; ++k)
            for (long long i = 0; i < L.ncell; ++i)
                h[(1 + k) * L.ncell + i] = d->u_init ? d->u_init[k * L.ncell + i] : d->u0[k];
        rc = upload_padded<T>(&c, c.init, h.data(), (int)nf);
        if (rc) return fail(err, rc, c.err);
    }
    long long mcount = L.ncell;
    if (has_mask) {
        std::vector<uint8_t> h(L.F, 0);
        mcount = 0;
        for (long long z = 0; z < L.g.n[2]; ++z)
            for (long long y = 0; y < L.g.n[1]; ++y)
                for (long long x = 0; x < L.g.n[0]; ++x) {
                    const uint8_t v = d->objective.mask[x + L.g.n[0] * (y + L.g.n[1] * z)] ? 1 : 0;
                    h[x + y * L.g.sy + z * L.g.sz] = v;
                    mcount += v;
                }
        he = hipMemcpy(c.mask, h.data(), L.F, hipMemcpyHostToDevice);
        if (he != hipSuccess) return fail(err, LKS_EDEVICE, hipGetErrorString(he));
    }
    c.d.rho_init = c.d.u_init = c.d.kappa_static = nullptr;
    c.d.objective.mask = nullptr;
    c.obj_scale = 1.0;
    if (d->objective.normalize & LKS_NORM_TIME) c.obj_scale /= (double)(d->objective.n1 - d->objective.n0 + 1);
    if (d->objective.normalize & LKS_NORM_MASK) c.obj_scale /= (double)std::max(1LL, mcount);

    rc = forward_impl<T>(&c, gamma, J);
    if (rc) return fail(err, rc, c.err);
    const size_t rows = (size_t)L.g.n[1] * L.g.n[2];
    if (drho) check(hipMemcpy2DAsync(drho, L.g.n[0] * e, c.fin, L.pitch * e, L.g.n[0] * e, rows,
                                     hipMemcpyDefault, c.stream));
    if (u)
        for (int k = 0; k < D; ++k)
            check(hipMemcpy2DAsync(static_cast<char *>(u) + (size_t)k * L.ncell * e, L.g.n[0] * e,
                                   c.field(c.fin, 1 + k), L.pitch * e, L.g.n[0] * e, rows, hipMemcpyDefault,
                                   c.stream));
    check(hipStreamSynchronize(c.stream));
    return rc;
}

}  // namespace

// ================================ continuous batching ========================================
// A batch advances many contexts by one micro-step each per round: one forward (or recompute)
// step, or one adjoint step plus its sensitivity gather.  The kernels of every context in the
// same micro-step kind share one launch over a (job, tile) list; per-job argument blocks are
// staged through a ring of pinned buffers so the host can run ahead of the device.
struct lks_batch {
    hipStream_t stream = nullptr;
    static constexpr int kSlots = 8;
    static constexpr size_t kCap = 4u << 20;
    char *host[kSlots] = {};
    char *dev[kSlots] = {};
    hipEvent_t ev[kSlots] = {};
    bool used[kSlots] = {};
    int next = 0;
    long rounds = 0;
    std::string err;
};

namespace {

enum { PH_IDLE = 0, PH_FWD = 1, PH_ADJ_BEGIN = 2, PH_ADJ = 3, PH_DONE = 6 };

template <typename T>
struct RoundLists {
    std::vector<lks::FwdArgs<T>> pre[3];   // transfer-only launches, before the forward launches
    std::vector<long long> ptiles[3];
    std::vector<lks::FwdArgs<T>> fwd[3];   // 2D, 3D D3Q19, 3D D3Q15
    std::vector<long long> ftiles[3];
    std::vector<lks::AdjArgs<T>> adj[3];
    std::vector<long long> atiles[3], ablk[3];
    std::vector<lks::SensArgs<T>> sens;
    std::vector<long long> sblk;
    struct Reduce {
        lks_ctx *c;
        int na, nb;
    };
    std::vector<Reduce> red;  // objective rows to reduce after this round's forward launches
    struct Scan {
        lks_ctx *c;
        const T *p, *q;
        int n, keep_max;
    };
    std::vector<Scan> scans;  // non-finite guards after this round's stencil launches
};

int list_of(const lks_ctx *c) { return c->d.dim == 2 ? 0 : (c->d.lattice == LKS_D3Q19 ? 1 : 2); }

long long adj_tiles(const lks_ctx *c) {
    if (c->d.dim == 2) return lks::tiles2d(c->L.g);
    return lks::tiles3d_adj(c->L.g, (int)c->L.esz);
}

template <typename T>
int begin_impl(lks_ctx *c, const void *gamma, void *out) {
    const Layout &L = c->L;
    const int D = c->d.dim;
    c->have_fwd = c->have_adj = false;
    HIPCHK(c, hipMemcpyAsync(c->gamma, gamma, L.nd * sizeof(T), hipMemcpyDefault, c->stream));
    HIPCHK(c, lks::launch_design_prep<T>(reinterpret_cast<const T *>(c->gamma),
                                         reinterpret_cast<T *>(c->kref), c->kprime, L.nd,
                                         c->d.interp == LKS_INTERP_PAPER ? 0 : 1,
                                         c->d.kappa_max, c->d.q, c->stream));
    HIPCHK(c, lks::launch_fill<double>(c->jn, 0.0, c->d.nsteps + 1, c->stream));
    if (int rc = reset_flags(c, true, c->stream)) return rc;
    Fields<T> st = state_fields<T>(c, c->state);
    lks::InitArgs<T> ia{};
    ia.g = L.g;
    ia.bc = bc_params<T>(c->d);
    ia.r0 = (T)(c->d.rho0 - 1.0);
    for (int k = 0; k < 3; ++k) ia.u0[k] = k < D ? (T)c->d.u0[k] : T(0);
    if (c->init) {
        Fields<T> in = state_fields<T>(c, c->init);
        ia.rinit = in.r;
        for (int k = 0; k < 3; ++k) ia.uinit[k] = in.u[k];
    }
    ia.rout = st.r;
    for (int k = 0; k < 3; ++k) ia.uout[k] = st.u[k];
    HIPCHK(c, lks::launch_init<T>(ia, c->stream));
    c->out_dev = out;
    c->cs = lks_ctx::Cursor{};
    c->cs.phase = PH_FWD;
    c->cs.n = 1;
    return LKS_OK;
}

// Enqueue this context's copies for its next micro-step and append its kernel arguments.
// Returns 1 if the forward sweep ends with this step, 2 if the reverse sweep does, else 0.
template <typename T>
int plan_step(lks_ctx *c, RoundLists<T> &R, int *rc) {
    const Layout &L = c->L;
    const int D = c->d.dim, N = c->d.nsteps, K = L.K, S = L.S;
    auto &cs = c->cs;
    Fields<T> st[2] = {state_fields<T>(c, c->state), state_fields<T>(c, c->field(c->state, 1 + D))};
    const int li = list_of(c);
    auto seg_lo = [&](int sg) { return sg * K + 1; };
    auto seg_hi = [&](int sg) { return std::min((sg + 1) * K, N); };
    *rc = LKS_OK;
    if (cs.phase == PH_FWD) {
        const int n = cs.n, seg = (n - 1) / K, j = n - seg * K;
        const bool last = seg == S - 1;
        if (j == 1) {
            T *ck = reinterpret_cast<T *>(c->field(c->ckpt, (long long)seg * (1 + D)));
            if ((*rc = copy_fields<T>(c, ck, st[cs.cur].r, 1))) return 0;
            if ((*rc = copy_fields<T>(c, ck + L.F, st[cs.cur].u[0], D))) return 0;
            if (last) {
                T *t0[3];
                traj_slot<T>(c, 0, 0, t0);
                if ((*rc = copy_fields<T>(c, t0[0], st[cs.cur].u[0], D))) return 0;
            }
        }
        T *uin[3], *uout[3];
        if (last) {
            traj_slot<T>(c, 0, j - 1, uin);
            traj_slot<T>(c, 0, j, uout);
        } else {
            for (int k = 0; k < 3; ++k) {
                uin[k] = st[cs.cur].u[k];
                uout[k] = st[1 - cs.cur].u[k];
            }
        }
        if (n == 1) {
            R.pre[li].push_back(make_xfer_args<T>(c, 1, fwd_loc<T>(c, 1)));
            R.ptiles[li].push_back(fwd_tiles(c, lks::FWD_TRANSFER_NEXT));
        }
        R.fwd[li].push_back(make_fwd_args<T>(c, n, st[cs.cur].r, uin, st[1 - cs.cur].r, uout, fwd_loc<T>(c, n),
                                             n < N ? fwd_loc<T>(c, n + 1) : nullptr, true));
        R.ftiles[li].push_back(fwd_tiles(c, R.fwd[li].back().mode));
        if (scan_fwd_step(c, n)) R.scans.push_back({c, R.fwd[li].back().rout, R.fwd[li].back().uout[0], n, 0});
        if (const int na = reduce_from(c, n)) R.red.push_back({c, na, n});
        cs.cur = 1 - cs.cur;
        cs.n = n + 1;
        return cs.n > N ? 1 : 0;
    }
    if (cs.phase == PH_ADJ_BEGIN) {
        Fields<T> ad = state_fields<T>(c, c->adj);
        HIPCHK(c, lks::launch_fill<T>(ad.r, T(0), (long long)(1 + D) * L.F, c->stream));
        HIPCHK(c, lks::launch_fill<double>(c->G, 0.0, L.nd, c->stream));
        cs.seg = S - 1;
        cs.n = seg_hi(cs.seg);
        cs.acur = 0;
        cs.ready = S - 1;  // lowest segment whose trajectory bank is complete (the forward wrote S-1)
        cs.rseg = -1;      // segment being recomputed, -1 when none
        cs.phase = PH_ADJ;
    }
    if (cs.phase == PH_ADJ) {
        // Reverse rounds: one recompute step of segment seg-1 (into the other bank) and one adjoint
        // step of segment seg, in the same round.  Segment seg-1 is restored once the adjoint of
        // seg+1, which used its bank, is done; the adjoint of a segment waits for its recompute.
        if (cs.rseg < 0 && cs.seg - 1 >= 0 && cs.seg - 1 < cs.ready) {
            cs.rseg = cs.seg - 1;
            const T *ck = reinterpret_cast<const T *>(c->field(c->ckpt, (long long)cs.rseg * (1 + D)));
            T *t0[3];
            traj_slot<T>(c, bank_of(c, cs.rseg), 0, t0);
            if ((*rc = copy_fields<T>(c, st[0].r, ck, 1))) return 0;
            if ((*rc = copy_fields<T>(c, t0[0], ck + L.F, D))) return 0;
            R.pre[li].push_back(make_xfer_args<T>(c, seg_lo(cs.rseg), rec_loc<T>(c, cs.rseg, seg_lo(cs.rseg))));
            R.ptiles[li].push_back(fwd_tiles(c, lks::FWD_TRANSFER_NEXT));
            cs.cur = 0;
            cs.rn = seg_lo(cs.rseg);
        }
        if (cs.rseg >= 0) {
            const int n = cs.rn, j = n - cs.rseg * K;
            T *uin[3], *uout[3];
            traj_slot<T>(c, bank_of(c, cs.rseg), j - 1, uin);
            traj_slot<T>(c, bank_of(c, cs.rseg), j, uout);
            R.fwd[li].push_back(make_fwd_args<T>(c, n, st[cs.cur].r, uin, st[1 - cs.cur].r, uout,
                                                 rec_loc<T>(c, cs.rseg, n),
                                                 n < seg_hi(cs.rseg) ? rec_loc<T>(c, cs.rseg, n + 1) : nullptr,
                                                 false));
            R.ftiles[li].push_back(fwd_tiles(c, R.fwd[li].back().mode));
            cs.cur = 1 - cs.cur;
            cs.rn = n + 1;
            if (cs.rn > seg_hi(cs.rseg)) {
                cs.ready = cs.rseg;
                cs.rseg = -1;
            }
        }
        if (cs.ready <= cs.seg) {
            const int n = cs.n, j = n - cs.seg * K;
            R.adj[li].push_back(make_adj_args<T>(c, n, j, cs.acur));
            if (scan_adj_step(n)) R.scans.push_back({c, R.adj[li].back().Pout, R.adj[li].back().Vout[0], n, 1});
            R.atiles[li].push_back(adj_tiles(c));
            R.ablk[li].push_back(lks::prep_blocks3(L.ncell));  // 3D pointwise adjoint blocks
            R.sens.push_back(make_sens_args<T>(c, n));
            R.sblk.push_back((L.nd + lks::kBlockHost - 1) / lks::kBlockHost);
            cs.acur = 1 - cs.acur;
            cs.n = n - 1;
            if (cs.n < seg_lo(cs.seg)) {
                cs.seg -= 1;
                if (cs.seg < 0) return 2;
                cs.n = seg_hi(cs.seg);
            }
        }
        return 0;
    }
    return 0;
}

template <typename T>
int end_forward(lks_ctx *c) {
    const Layout &L = c->L;
    const int D = c->d.dim, N = c->d.nsteps, K = L.K, S = L.S;
    Fields<T> st = state_fields<T>(c, c->field(c->state, (long long)c->cs.cur * (1 + D)));
    Fields<T> fin = state_fields<T>(c, c->fin);
    T *ul[3];
    traj_slot<T>(c, 0, N - (S - 1) * K, ul);
    int rc;
    if ((rc = copy_fields<T>(c, fin.r, st.r, 1))) return rc;
    if ((rc = copy_fields<T>(c, fin.u[0], ul[0], D))) return rc;
    HIPCHK(c, hipMemcpyAsync(c->jn_host, c->jn, (N + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    c->cs.phase = PH_ADJ_BEGIN;
    return LKS_OK;
}

template <typename T>
int end_reverse(lks_ctx *c) {
    HIPCHK(c, lks::launch_sens_finish<T>(c->kprime, c->G, reinterpret_cast<T *>(c->out_dev), c->L.nd, c->stream));
    HIPCHK(c, lks::launch_scan<double>(c->G, c->L.nd, nullptr, 0, 1, c->flag + 2, 1, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->flag_host, c->flag, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipEventRecord(c->done_ev, c->stream));
    c->cs.phase = PH_DONE;
    return LKS_OK;
}

size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

template <typename T>
int round_impl(lks_batch *b, lks_ctx *const *cs, int n, int *done) {
    RoundLists<T> R;
    std::vector<int> ends(n, 0);
    for (int i = 0; i < n; ++i) {
        int rc = LKS_OK;
        ends[i] = plan_step<T>(cs[i], R, &rc);
        if (rc) {
            b->err = cs[i]->err;
            return rc;
        }
    }
    // stage every argument list into one pinned slot and one device copy
    const int sl = b->next;
    b->next = (b->next + 1) % lks_batch::kSlots;
    if (b->used[sl] && hipEventSynchronize(b->ev[sl]) != hipSuccess) {
        b->err = "staging event failed";
        return LKS_EDEVICE;
    }
    char *h = b->host[sl];
    size_t off = 0;
    auto put = [&](const void *src, size_t bytes) -> long long {
        const size_t o = off;
        if (off + align_up(bytes) > lks_batch::kCap) return -1;
        if (bytes) std::memcpy(h + off, src, bytes);
        off += align_up(bytes);
        return (long long)o;
    };
    auto prefix = [](const std::vector<long long> &v, std::vector<long long> &p) {
        p.resize(v.size());
        long long acc = 0;
        for (size_t i = 0; i < v.size(); ++i) {
            p[i] = acc;
            acc += v[i];
        }
        return acc;
    };
    struct Launch {
        int kind, li;
        long long args, t0, t1, total, total1;
        int njobs;
        bool pz = false;  // 3D: every job of the launch periodic in z
    };
    std::vector<Launch> ls;
    for (int li = 0; li < 3; ++li) {
        if (!R.pre[li].empty()) {
            std::vector<long long> p;
            const long long tot = prefix(R.ptiles[li], p);
            Launch L{0, li, put(R.pre[li].data(), R.pre[li].size() * sizeof(lks::FwdArgs<T>)),
                     put(p.data(), p.size() * 8), 0, tot, 0, (int)R.pre[li].size()};
            L.pz = true;
            for (const auto &fj : R.pre[li]) L.pz = L.pz && fj.g.per[2] != 0;
            ls.push_back(L);
        }
    }
    for (int li = 0; li < 3; ++li) {
        if (!R.fwd[li].empty()) {
            std::vector<long long> p;
            const long long tot = prefix(R.ftiles[li], p);
            Launch L{0, li, put(R.fwd[li].data(), R.fwd[li].size() * sizeof(lks::FwdArgs<T>)),
                     put(p.data(), p.size() * 8), 0, tot, 0, (int)R.fwd[li].size()};
            L.pz = true;
            for (const auto &fj : R.fwd[li]) L.pz = L.pz && fj.g.per[2] != 0;
            ls.push_back(L);
        }
        if (!R.adj[li].empty()) {
            std::vector<long long> p, q;
            const long long tot = prefix(R.atiles[li], p);
            const long long totb = prefix(R.ablk[li], q);
            Launch L{1, li, put(R.adj[li].data(), R.adj[li].size() * sizeof(lks::AdjArgs<T>)),
                     put(p.data(), p.size() * 8), put(q.data(), q.size() * 8), tot, totb,
                     (int)R.adj[li].size()};
            L.pz = true;
            for (const auto &aj : R.adj[li]) L.pz = L.pz && aj.g.per[2] != 0;
            ls.push_back(L);
        }
    }
    if (!R.sens.empty()) {
        std::vector<long long> p;
        const long long tot = prefix(R.sblk, p);
        Launch L{2, 0, put(R.sens.data(), R.sens.size() * sizeof(lks::SensArgs<T>)),
                 put(p.data(), p.size() * 8), 0, tot, 0, (int)R.sens.size()};
        ls.push_back(L);
    }
    for (const Launch &L : ls)
        if (L.args < 0 || L.t0 < 0 || L.t1 < 0) {
            b->err = "too many jobs in one round for the staging buffer";
            return LKS_EINVAL;
        }
    if (off) {
        hipError_t e = hipMemcpyAsync(b->dev[sl], h, off, hipMemcpyHostToDevice, b->stream);
        if (e != hipSuccess) {
            b->err = hipGetErrorString(e);
            return LKS_EDEVICE;
        }
    }
    char *dv = b->dev[sl];
    for (const Launch &L : ls) {
        hipError_t e = hipSuccess;
        const auto *t0 = reinterpret_cast<const long long *>(dv + L.t0);
        if (L.kind == 0) {
            const auto *a = reinterpret_cast<const lks::FwdArgs<T> *>(dv + L.args);
            e = L.li == 0 ? lks::launch_fwd2d_batch<T>(a, t0, L.njobs, L.total, b->stream)
                          : lks::launch_fwd3d_batch<T>(a, t0, L.njobs, L.total, L.li == 1 ? LKS_D3Q19 : LKS_D3Q15, L.pz,
                                                       b->stream);
        } else if (L.kind == 1) {
            const auto *a = reinterpret_cast<const lks::AdjArgs<T> *>(dv + L.args);
            e = L.li == 0 ? lks::launch_adj2d_batch<T>(a, t0, L.njobs, L.total, b->stream)
                          : lks::launch_adj3d_batch<T>(a, reinterpret_cast<const long long *>(dv + L.t1), L.total1,
                                                       t0, L.total, L.njobs, L.li == 1 ? LKS_D3Q19 : LKS_D3Q15, L.pz,
                                                       b->stream);
        }
        if (e != hipSuccess) {
            b->err = hipGetErrorString(e);
            return LKS_EDEVICE;
        }
    }
    for (const auto &r : R.red) {
        hipError_t e = lks::launch_reduce_steps(r.c->partials, r.c->L.max_blocks, r.c->L.max_blocks, r.na, r.nb,
                                                r.c->obj_scale, r.c->jn, b->stream);
        if (e != hipSuccess) {
            b->err = hipGetErrorString(e);
            return LKS_EDEVICE;
        }
    }
    for (const auto &sc : R.scans) {
        hipError_t e = lks::launch_scan<T>(sc.p, sc.c->L.F, sc.q, (long long)sc.c->d.dim * sc.c->L.F, sc.n,
                                           sc.c->flag + sc.keep_max, sc.keep_max, b->stream);
        if (e != hipSuccess) {
            b->err = hipGetErrorString(e);
            return LKS_EDEVICE;
        }
    }
    for (const Launch &L : ls) {  // sensitivity gathers after every adjoint step of the round
        if (L.kind != 2) continue;
        hipError_t e = lks::launch_sens_batch<T>(reinterpret_cast<const lks::SensArgs<T> *>(dv + L.args),
                                                 reinterpret_cast<const long long *>(dv + L.t0), L.njobs,
                                                 L.total, b->stream);
        if (e != hipSuccess) {
            b->err = hipGetErrorString(e);
            return LKS_EDEVICE;
        }
    }
    if (hipEventRecord(b->ev[sl], b->stream) != hipSuccess) {
        b->err = "event record failed";
        return LKS_EDEVICE;
    }
    b->used[sl] = true;
    for (int i = 0; i < n; ++i) {
        int rc = LKS_OK;
        if (ends[i] == 1) rc = end_forward<T>(cs[i]);
        else if (ends[i] == 2) rc = end_reverse<T>(cs[i]);
        if (rc) {
            b->err = cs[i]->err;
            return rc;
        }
        if (done) done[i] = cs[i]->cs.phase == PH_DONE;
    }
    b->rounds++;
    return LKS_OK;
}

}  // namespace

namespace {
int set_err(lks_ctx *c, int code, const char *msg) {
    if (c) c->err = msg;
    return code;
}

}  // namespace

// ====================================== C ABI ===============================================
extern "C" {

int lks_query_bytes(const lks_desc *d, size_t *bytes) {
    Layout L;
    std::string err;
    int rc = plan(d, L, &err);
    if (rc == LKS_ENOMEM && bytes) {
        *bytes = L.bytes;
        return LKS_OK;
    }
    if (rc) {
        g_create_error = err;
        return rc;
    }
    if (!bytes) return LKS_EINVAL;
    *bytes = L.bytes;
    return LKS_OK;
}

int lks_create(const lks_desc *d, lks_ctx **out) {
    if (!out) {
        g_create_error = "out is NULL";
        return LKS_EINVAL;
    }
    *out = nullptr;
    lks_ctx *c = new (std::nothrow) lks_ctx();
    if (!c) {
        g_create_error = "host allocation failed";
        return LKS_ENOMEM;
    }
    int rc = plan(d, c->L, &g_create_error);
    if (rc == LKS_OK) rc = create_impl(d, c);
    if (rc != LKS_OK) {
        if (!c->err.empty()) g_create_error = c->err;
        lks_destroy(c);
        return rc;
    }
    *out = c;
    return LKS_OK;
}

void lks_destroy(lks_ctx *c) {
    if (!c) return;
    if (c->stream || !c->allocs.empty()) (void)hipStreamSynchronize(c->stream);
    if (c->stream2) {
        (void)hipStreamSynchronize(c->stream2);
        (void)hipStreamDestroy(c->stream2);
    }
    for (hipEvent_t e : {c->ev_fork, c->ev_rec, c->ev_adj})
        if (e) (void)hipEventDestroy(e);
    for (void *p : c->allocs) (void)hipFree(p);
    for (auto &ev : c->pool) {
        if (ev.a) (void)hipEventDestroy(ev.a);
        if (ev.b) (void)hipEventDestroy(ev.b);
    }
    if (c->done_ev) (void)hipEventDestroy(c->done_ev);
    if (c->jn_host) (void)hipHostFree(c->jn_host);
    if (c->arghost) (void)hipHostFree(c->arghost);
    if (c->flag_host) (void)hipHostFree(c->flag_host);
    delete c;
}

int lks_forward(lks_ctx *c, const void *gamma, double *J) {
    if (!c) return LKS_EINVAL;
    if (!gamma) return set_err(c, LKS_EINVAL, "gamma is NULL");
    try {
        return c->L.esz == 8 ? forward_impl<double>(c, gamma, J) : forward_impl<float>(c, gamma, J);
    } catch (...) {
        return set_err(c, LKS_ENOMEM, "host exception in lks_forward");
    }
}

int lks_forward_noalloc(const lks_desc *d, const void *gamma, double *J, void *drho, void *u) {
    if (!d || !gamma) {
        g_create_error = "descriptor or gamma is NULL";
        return LKS_EINVAL;
    }
    try {
        return d->precision == LKS_F64 ? forward_noalloc_impl<double>(d, gamma, J, drho, u, &g_create_error)
                                       : forward_noalloc_impl<float>(d, gamma, J, drho, u, &g_create_error);
    } catch (...) {
        g_create_error = "host exception in lks_forward_noalloc";
        return LKS_ENOMEM;
    }
}

int lks_adjoint(lks_ctx *c) {
    if (!c) return LKS_EINVAL;
    if (c->L.fwd_only) return set_err(c, LKS_ESTATE, "the objective is NONE: nothing to differentiate");
    if (!c->have_fwd) return set_err(c, LKS_ESTATE, "lks_adjoint needs a successful lks_forward first");
    try {
        return c->L.esz == 8 ? adjoint_impl<double>(c) : adjoint_impl<float>(c);
    } catch (...) {
        return set_err(c, LKS_ENOMEM, "host exception in lks_adjoint");
    }
}

int lks_sensitivity(lks_ctx *c, void *dJdgamma) {
    if (!c) return LKS_EINVAL;
    if (!dJdgamma) return set_err(c, LKS_EINVAL, "output is NULL");
    if (!c->have_adj) return set_err(c, LKS_ESTATE, "lks_sensitivity needs lks_adjoint after the last lks_forward");
    const long long nd = c->L.nd;
    hipError_t e = c->L.esz == 8
        ? lks::launch_sens_finish<double>(c->kprime, c->G, reinterpret_cast<double *>(c->sens), nd, c->stream)
        : lks::launch_sens_finish<float>(c->kprime, c->G, reinterpret_cast<float *>(c->sens), nd, c->stream);
    HIPCHK(c, e);
    HIPCHK(c, hipMemcpyAsync(dJdgamma, c->sens, nd * c->L.esz, hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LKS_OK;
}

int lks_read_state(lks_ctx *c, int which, void *drho, void *u) {
    if (!c) return LKS_EINVAL;
    if (!c->have_fwd) return set_err(c, LKS_ESTATE, "no forward state yet");
    const Layout &L = c->L;
    const int D = c->d.dim;
    char *base;
    if (which == LKS_STATE_FINAL) base = c->fin;
    else if (which >= 0 && which < L.S && (L.S > 1 || which == 0)) base = c->field(c->ckpt, (long long)which * (1 + D));
    else return set_err(c, LKS_EINVAL, "unknown state index");
    const size_t e = L.esz;
    const size_t rows = (size_t)L.g.n[1] * L.g.n[2];
    if (drho)
        HIPCHK(c, hipMemcpy2DAsync(drho, L.g.n[0] * e, base, L.pitch * e, L.g.n[0] * e, rows,
                                   hipMemcpyDefault, c->stream));
    if (u)
        for (int k = 0; k < D; ++k)
            HIPCHK(c, hipMemcpy2DAsync(static_cast<char *>(u) + (size_t)k * L.ncell * e, L.g.n[0] * e,
                                       c->field(base, 1 + k), L.pitch * e, L.g.n[0] * e, rows,
                                       hipMemcpyDefault, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LKS_OK;
}

int lks_read_objective_steps(lks_ctx *c, double *jn) {
    if (!c || !jn) return LKS_EINVAL;
    if (!c->have_fwd) return set_err(c, LKS_ESTATE, "no forward yet");
    HIPCHK(c, hipMemcpyAsync(jn, c->jn, (c->d.nsteps + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LKS_OK;
}

int lks_set_timing(lks_ctx *c, int every) {
    if (!c || every < 0) return LKS_EINVAL;
    int rc = flush_timing(c);
    if (rc) return rc;
    c->every = every;
    for (int k = 0; k < 3; ++k) c->launches[k] = c->samples[k] = 0, c->total_ms[k] = 0;
    if (every > 0 && c->pool.empty()) {
        c->pool.resize(512);
        // device-scope events: no system-wide cache release around the timed kernel
        for (auto &ev : c->pool) {
            if (hipEventCreateWithFlags(&ev.a, hipEventDisableSystemFence) != hipSuccess)
                HIPCHK(c, hipEventCreate(&ev.a));
            if (hipEventCreateWithFlags(&ev.b, hipEventDisableSystemFence) != hipSuccess)
                HIPCHK(c, hipEventCreate(&ev.b));
        }
    }
    return LKS_OK;
}

int lks_kernel_timing(lks_ctx *c, int kind, long *count, double *mean_ms) {
    if (!c || kind < 0 || kind > 2) return LKS_EINVAL;
    int rc = flush_timing(c);
    if (rc) return rc;
    if (count) *count = c->samples[kind];
    if (mean_ms) *mean_ms = c->samples[kind] ? c->total_ms[kind] / c->samples[kind] : 0.0;
    (void)kind_name;
    return LKS_OK;
}

int lks_batch_create(void *stream, lks_batch **out) {
    if (!out) return LKS_EINVAL;
    *out = nullptr;
    lks_batch *b = new (std::nothrow) lks_batch();
    if (!b) return LKS_ENOMEM;
    b->stream = reinterpret_cast<hipStream_t>(stream);
    for (int i = 0; i < lks_batch::kSlots; ++i) {
        if (hipHostMalloc(reinterpret_cast<void **>(&b->host[i]), lks_batch::kCap, 0) != hipSuccess ||
            hipMalloc(reinterpret_cast<void **>(&b->dev[i]), lks_batch::kCap) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) {
            g_create_error = "batch staging allocation failed";
            lks_batch_destroy(b);
            return LKS_ENOMEM;
        }
    }
    *out = b;
    return LKS_OK;
}

void lks_batch_destroy(lks_batch *b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (int i = 0; i < lks_batch::kSlots; ++i) {
        if (b->host[i]) (void)hipHostFree(b->host[i]);
        if (b->dev[i]) (void)hipFree(b->dev[i]);
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
    }
    delete b;
}

int lks_begin(lks_ctx *c, const void *gamma, void *dJdgamma) {
    if (c && c->d.adjoint_form != LKS_ADJ_EXACT)
        return set_err(c, LKS_EUNSUPPORTED, "the served path runs the exact adjoint only");
    if (!c) return LKS_EINVAL;
    if (!gamma || !dJdgamma) return set_err(c, LKS_EINVAL, "gamma and dJdgamma are required");
    if (!c->d.io_on_device) return set_err(c, LKS_EINVAL, "lks_begin needs an io_on_device context");
    if (c->L.fwd_only) return set_err(c, LKS_ESTATE, "the objective is NONE: nothing to differentiate");
    if (c->cs.phase != 0 && c->cs.phase != 6) return set_err(c, LKS_ESTATE, "an evaluation is in flight");
    if (!c->jn_host) {
        if (hipHostMalloc(reinterpret_cast<void **>(&c->jn_host), (c->d.nsteps + 1) * sizeof(double), 0) != hipSuccess ||
            hipHostMalloc(reinterpret_cast<void **>(&c->flag_host), 3 * sizeof(int), 0) != hipSuccess ||
            hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess)
            return set_err(c, LKS_ENOMEM, "pinned host allocation failed");
    }
    try {
        return c->L.esz == 8 ? begin_impl<double>(c, gamma, dJdgamma) : begin_impl<float>(c, gamma, dJdgamma);
    } catch (...) {
        return set_err(c, LKS_ENOMEM, "host exception in lks_begin");
    }
}

int lks_batch_round(lks_batch *b, lks_ctx *const *cs, int n, int *done) {
    if (!b || (n > 0 && !cs)) return LKS_EINVAL;
    if (n == 0) return LKS_OK;
    const size_t esz = cs[0]->L.esz;
    for (int i = 0; i < n; ++i) {
        if (!cs[i] || cs[i]->L.esz != esz || cs[i]->stream != b->stream) {
            b->err = "every context of a round needs the batch stream and the same precision";
            return LKS_EINVAL;
        }
        if (cs[i]->cs.phase == 0) {
            b->err = "context has no evaluation in flight (call lks_begin)";
            return LKS_ESTATE;
        }
    }
    try {
        return esz == 8 ? round_impl<double>(b, cs, n, done) : round_impl<float>(b, cs, n, done);
    } catch (...) {
        b->err = "host exception in lks_batch_round";
        return LKS_ENOMEM;
    }
}

const char *lks_batch_error(const lks_batch *b) { return b ? b->err.c_str() : "NULL batch"; }

int lks_poll(lks_ctx *c) {
    if (!c) return LKS_EINVAL;
    if (c->cs.phase != 6) return 0;
    const hipError_t e = hipEventQuery(c->done_ev);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    c->err = hipGetErrorString(e);
    return LKS_EDEVICE;
}

int lks_finish(lks_ctx *c, double *J) {
    if (!c) return LKS_EINVAL;
    if (c->cs.phase != 6) return set_err(c, LKS_ESTATE, "evaluation not finished");
    HIPCHK(c, hipEventSynchronize(c->done_ev));
    double acc = 0.0;
    for (int n = 0; n <= c->d.nsteps; ++n) acc += c->jn_host[n];
    if (J) *J = acc;
    c->cs.phase = 0;
    if (int rc = nonfinite_error(c, c->flag_host)) return rc;
    c->have_fwd = c->have_adj = true;
    return LKS_OK;
}

const char *lks_last_error(const lks_ctx *c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

const char *lks_strerror(int code) {
    switch (code) {
    case LKS_OK: return "ok";
    case LKS_EINVAL: return "invalid argument";
    case LKS_ENOMEM: return "out of memory or over the HBM budget";
    case LKS_ESTATE: return "call out of order";
    case LKS_ENONFINITE: return "non-finite state";
    case LKS_EDEVICE: return "HIP runtime error";
    case LKS_EUNSUPPORTED: return "unsupported";
    }
    return "unknown error";
}

}  // extern "C"

// Internal structures shared by the host runtime and the HIP kernels of the LKS library.
// Nothing here is part of the C ABI (include/lks.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lks {

// Analysis grid: node (x, y, z) lives at x + y*sy + z*sz in every field (rows padded).
struct Geom {
    int dim;
    int n[3];
    int per[3];        // 1 if the axis is periodic (always 1 for axes >= dim)
    long long sy, sz;  // element strides
    int zc;            // 3D: z planes marched per block of the forward (chosen at create)
    int zca;           // 3D: z planes marched per block of the z-marching adjoint
};

// Boundary kinds per face (x-, x+, y-, y+, z-, z+); rho is stored as rho - 1.
template <typename T>
struct BCParams {
    int kind[6];
    T rho[6];
    T u[6][3];
};

// Rigid motion at one step plus the footprint box of the mapped design grid (inclusive bounds).
struct StepMotion {
    double R[9];
    double Om[3];
    double xG[3];
    double uG[3];
    int lo[3];
    int hi[3];
};

template <typename T>
struct Design {
    const T *kref;  // kappa_ref on the design grid
    int nd[3];
    double xiG[3];
    int weight;     // 0 = COS4, 1 = LIN
};

// Footprint box store: fixed extent bn (max over steps), element strides.
struct BoxGeom {
    int bn[3];
    long long bsy, bsz, cells;
};

struct ObjParams {
    int kind;          // LKS_OBJ_* (-1 none)
    int active;        // this step lies in the window
    double scale;      // 1/(n1-n0+1) and/or 1/|mask|
    double centre[3];
    double dir[3];
    const uint8_t *mask;    // padded like the fields, or null
    double *partials;       // this step's row of per-block partials
};

template <typename T>
struct FwdArgs {
    Geom g;
    BCParams<T> bc;
    T A;
    T gf[3];
    const T *rin;
    const T *uin[3];
    T *rout;
    T *uout[3];
    const T *kstatic;
    Design<T> des;
    StepMotion m;
    BoxGeom box;
    const T *kin;       // kappa and u_S of this step on its footprint box
    const T *usin[3];
    int mode;           // bit 0: run the stencil; bit 1: transfer the next step
    StepMotion mnext;   // motion of the step transferred by the extra blocks
    T *knext;           // where the extra blocks write the next step's kappa and u_S
    T *usnext[3];
    ObjParams obj;
    const void *next;   // 2D: argument block of the sweep's next step (this launch prefetches it), or null
};
// FWD_TRANSFER_FIRST (2D): the transfer blocks precede the stencil tiles in the launch
enum { FWD_STENCIL = 1, FWD_TRANSFER_NEXT = 2, FWD_TRANSFER_FIRST = 4 };

template <typename T>
struct SensArgs;

template <typename T>
struct AdjArgs {
    Geom g;
    BCParams<T> bc;
    T A;
    const T *Pin;
    const T *Vin[3];
    T *Pout;
    T *Vout[3];
    const T *uprev[3];  // input velocity of the forward step
    const T *ucur[3];   // output velocity of the forward step
    const T *kstatic;
    const T *kbox;      // kappa and u_S of this step on the footprint box
    const T *usbox[3];
    T *kbar;            // adjoint of kappa on the footprint box (written)
    BoxGeom box;
    StepMotion m;
    ObjParams obj;
    T *Ps;              // 3D only: (P*, V*) scratch fields between the two adjoint kernels
    T *Vs[3];
    const SensArgs<T> *sens;  // 2D: gather of the previous adjoint step run by extra blocks, or null
    long long sens_blocks;
    // the paper's adjoint form (2D): 3 u~ of the level being left and of the new one, and the
    // s~ fields (xx, xy, yy) between the moment and strain launches; Ps / Vs hold (P*, V*)
    const T *U3in[3];
    T *U3out[3];
    T *st[3];
    const void *next;   // 2D: argument block of the sweep's next step (this launch prefetches it), or null
};

template <typename T>
struct SensArgs {
    const T *kbar;
    BoxGeom box;
    StepMotion m;
    Design<T> des;
    int dim;
    double *G;
};

template <typename T>
struct InitArgs {
    Geom g;
    BCParams<T> bc;
    T r0;
    T u0[3];
    const T *rinit;     // optional padded fields
    const T *uinit[3];
    T *rout;
    T *uout[3];
};

// bytes of argument blocks one time step of one context needs (forward + recompute + adjoint
// + gather)
template <typename T>
constexpr size_t args_bytes() {
    return 2 * sizeof(FwdArgs<T>) + sizeof(AdjArgs<T>) + sizeof(SensArgs<T>);
}

// ---- launchers (defined in the .hip files) -----------------------------------------------
template <typename T> hipError_t launch_init(const InitArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_design_prep(const T *gamma, T *kref, double *kprime, long long nd, int interp,
                              double kmax, double q, hipStream_t s);
template <typename T>
hipError_t launch_sens_finish(const double *kprime, const double *G, T *out, long long nd,
                              hipStream_t s);
template <typename T>
hipError_t launch_fill(T *p, T v, long long count, hipStream_t s);
// a NaN/Inf among p[0, np) and q[0, nq) sets *flag = min(*flag, step) (keep_max = 0) or
// max(*flag, step) (keep_max = 1)
template <typename T>
hipError_t launch_scan(const T *p, long long np, const T *q, long long nq, int step, int *flag, int keep_max,
                       hipStream_t s);
// the state of a sweep is scanned for NaN/Inf after every kScanEvery-th step (and the last)
constexpr int kScanEvery = 64;
// jn[n] = scale * sum_{b < nblocks} partials[(n - n0) * stride + b] for n in [n0, n1]
hipError_t launch_reduce_steps(const double *partials, long long stride, long long nblocks, int n0,
                               int n1, double scale, double *jn, hipStream_t s);

// batched launches: job j owns flat blocks [tile0[j], tile0[j+1]) (tile0 ascending from 0)
template <typename T>
hipError_t launch_fwd2d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, hipStream_t s);
template <typename T>
hipError_t launch_adj2d_batch(const AdjArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, hipStream_t s);
// pz: every job of the launch is periodic in z (three-plane velocity ring)
template <typename T>
hipError_t launch_fwd3d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs,
                              long long ntiles, int lattice, bool pz, hipStream_t s);
template <typename T>
hipError_t launch_xfer3d_batch(const FwdArgs<T> *args, const long long *tile0, int njobs, long long ntiles,
                               hipStream_t s);
template <typename T>
// pz: every job of the launch is periodic in z (smaller LDS layout of the z-marching kernel)
hipError_t launch_adj3d_batch(const AdjArgs<T> *args, const long long *blk0, long long nblk,
                              const long long *tile0, long long ntiles, int njobs, int lattice, bool pz,
                              hipStream_t s);
// the paper's adjoint step in 2D: three launches (prep, moments, strain) of one job
template <typename T>
hipError_t launch_padj2d(const AdjArgs<T> *args, const Geom &g, hipStream_t s);
template <typename T>
hipError_t launch_sens_batch(const SensArgs<T> *args, const long long *blk0, int njobs, long long nblk,
                             hipStream_t s);
long long tiles2d(const Geom &g);      // adjoint tiles
long long tiles2d_fwd(const Geom &g);  // forward blocks (four wave strips each)
long long tiles3d(const Geom &g, int esz);
// blocks a forward launch appends to transfer the next step onto a box of `cells` cells
long long xfer_blocks(int dim, long long cells, int esz);
long long xfer_blocks3d(long long cells, int esz);

// grid sizes of the stencil launches (used by the host to size the partials buffer)
long long fwd_blocks(const Geom &g, int lattice, int esz);
long long fwd_blocks3d(const Geom &g, int lattice, int esz);
int choose_zc3(const Geom &g, int esz);   // z planes per block of the 3D forward
int choose_zca3(const Geom &g, int esz);  // ... of the z-marching adjoint (after zc is set)
long long tiles3d_adj(const Geom &g, int esz);

// 64-node segments per wave of the 3D pointwise adjoint kernel: up to 8 where the grid still gives
// at least 8192 waves (about one per wave slot of the chip), fewer on smaller grids, at least 1
__host__ __device__ inline int prep_rows3(long long ncell) {
    const long long r = ncell / (64LL * 8192);
    return r < 1 ? 1 : (r > 8 ? 8 : (int)r);
}
// its grid: 256-thread blocks of four waves
__host__ __device__ inline long long prep_blocks3(long long ncell) {
    const long long per = 256LL * prep_rows3(ncell);
    return (ncell + per - 1) / per;
}

}  // namespace lks

// Kernel launch interface shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "hweno_device.h"

namespace hw {

// Pointers into the workspace are read by the kernels from device memory
// (the grid descriptors), where the compiler cannot tell their address space
// and would access them with flat instructions.  In the device pass they are
// typed as global-memory pointers, so the kernels use global loads and
// stores, whose completion is tracked per instruction (flat accesses also
// count against the LDS counter, which forces coarser waits).  Host code sees
// plain pointers; the layout is the same.
#if defined(__HIP_DEVICE_COMPILE__)
#define HW_GLOBAL __attribute__((address_space(1)))
#else
#define HW_GLOBAL
#endif
using gdouble = HW_GLOBAL double;

// Device-side reduction slots, one set per grid.  Doubles are stored as
// order-preserving keys (dkey) so that atomicMax / atomicMin work for any sign.
struct Reduce {
    unsigned long long alpha_key;     // max |u_n| + c over interior face traces
    unsigned long long beta_key;      // max LF coefficient over interior faces
    unsigned long long pp_cells;      // cells where the limiter acted (any stage)
    unsigned long long min_rho_key;   // min cell-average density (per call)
    unsigned long long min_p_key;     // min cell-average pressure
    unsigned int bad[4];              // inadmissible cells per stage (index 1..3)
    double dt;                        // step size used by the update kernels
    unsigned long long alpha1_key;    // alpha of the stage-1 reconstruction (copied by k_dt)
    double pad[2];
};

// Ghost-fill description of one side (xlo, xhi, ylo, yhi).
struct Side {
    int kind;             // HWENO_BC_* value
    double sign[12];      // multiplier per (moment, component) for walls
    double inflow[4];     // conservative inflow state
    const gdouble* prof;   // inflow profile: conservative state of boundary cell k at
                          // prof[4 k .. 4 k + 3] (rows of an x side, columns of a y
                          // side); null: the constant state above
    const gdouble* prof_stage;   // profiles of the three RK stages, n cells each
                                // (stage s, cell k at 4 (s n + k)); used only by
                                // ghost fills that name a stage
};

// Persistent per-instance state of a batched run (device memory).  Kernels
// of the 2D pipeline skip every instance whose `active` is 0.
struct InstState {
    double t, t_final;        // time; end time (<= 0: none)
    double cfl_h, visc_dt;    // step rule: min(cfl_h / alpha*, visc_dt, t_final - t)
    double dt_last;           // step size of the last accepted step
    double alpha, beta_max, min_rho, min_p;   // diagnostics of the last attempt
    unsigned long long restarts;   // rejected attempts in this run
    unsigned long long pp_cells;   // limiter cell-stages of accepted steps in this run
    int steps, target;        // accepted steps in this run and the goal
    int halvings, max_halvings;
    int active;               // 1 while steps < target, t < t_final and no error
    int status;               // 0, or the hweno_status that stopped the instance
};

// Compact volume data per basis: the convective flux sum and the point
// velocities and viscosities the gradient kernel's viscous volume flux needs.
constexpr int VC_B = 31;

// Pointers and sizes of one 2D grid's workspace (all arrays SoA over the
// ghosted grid NX x NY, component-major: a[q * ncell + j * NX + i]).
struct Grid2 {
    int nx, ny, NX, NY;       // interior and ghosted sizes (halo 4)
    long long ncell;          // NX * NY
    Consts K;
    Side side[4];
    gdouble* S[4];  // 12 each: ghosted states (current, stage outputs, scratch)
    HW_GLOBAL InstState* st;
    gdouble* xf;   // 24: x-face traces (p*4 + c), p 0..2 left face, 3..5 right face
    gdouble* yf;   // 24: y-face traces, p 0..2 bottom face, 3..5 top face
    gdouble* xv;   // 36: x-basis volume values (q*4 + c), q = 3*h + g; written only
                   // for the reverse mode (full_grad), which reads them
    gdouble* yv;   // 36: y-basis volume values (likewise)
    gdouble* vc;   // 2 * VC_B: per basis b (x for f, y for g), at b * VC_B: the
                   // Gauss sum of the convective flux (4), then u, v and mu at
                   // the nine volume points (9 each; mu only with mu(T))
    gdouble* wb;   // 6:  wbar of (u, v, e) from x-basis, then from y-basis
    gdouble* vk;   // 8:  modified moments of the current input (hat-v 0..3, hat-w 4..7)
    gdouble* vn;   // 8:  modified moments of U^n (kept for stages 2 and 3)
    gdouble* rb;   // 18: weak moments ((l*3 + w)*3 + mom)
    gdouble* gf;   // gradients at the face points, p 0..5 x-face, 6..11 y-face: 36, the
                   // three combinations of stress_combos (p*3 + z), or with the
                   // reverse mode's full_grad 72, the six gradients (p*6 + s)
    gdouble* vf;   // 8:  volume flux quadratures (sum f, sum g)
    gdouble* fx;   // 8: x-face flux moments at (j, i+1/2): sum_G w_G F (c), sum_G w_G x_G F (4 + c)
    gdouble* fy;   // 8: y-face flux moments at (j+1/2, i)
    HW_GLOBAL Reduce* red;
    // masked domain (single grid): interior mask (1 = solid, j*nx + i) or null;
    // solid cells next to the fluid: ghosted destination, ghosted mirror source
    // and wall direction (0: x face, 1: y face); wall kind (slip or no-slip)
    const HW_GLOBAL unsigned char* solid;
    const HW_GLOBAL int* sdst;
    const HW_GLOBAL int* ssrc;
    const HW_GLOBAL int* sdir;
    int nsolid;
    int solid_wall;
    double fixed_state[4];   // conservative state of the solid cells listed with source -1
};

struct Grid1 {
    int nx, NX;               // interior and ghosted (halo 4) sizes
    Consts K;
    Side side[2];
    gdouble* pts;  // 12: limited LGL point values (p*3 + c)
    gdouble* wb;   // 2: wbar of (u, e)
    gdouble* vk;   // 3: modified moment of the current input
    gdouble* vn;   // 3: modified moment of U^n
    gdouble* rb;   // 4: weak moments (w*2 + mom)
    gdouble* gr;   // 8: gradients at the LGL points (p*2 + w)
    gdouble* fh;   // 3: face flux at i+1/2
    gdouble* vf;   // 3: volume flux quadrature
    HW_GLOBAL Reduce* red;
};

// Optional per-kernel timing with HIP events on the launch stream.  Kernel
// classes: 0 ghost, 1 recon, 2 rbar, 3 grad, 4 flux, 5 update, 6 other,
// 7 face fluxes fused with the update.
enum { KC_GHOST = 0, KC_RECON, KC_RBAR, KC_GRAD, KC_FLUX, KC_UPDATE, KC_OTHER, KC_FLUXUP,
       KC_COUNT };

struct Timer {
    static constexpr int CAP = 1024;
    bool on = false;
    bool ready = false;
    bool open = false;          // a begin() was recorded and awaits its end()
    unsigned mask = 0;          // kernel classes recorded (bit k = class k)
    int n = 0;
    int cls[CAP];
    hipEvent_t a[CAP], b[CAP];
    double ms[KC_COUNT];
    unsigned long long launches[KC_COUNT];
    bool init() {
        if (ready) return true;
        for (int i = 0; i < CAP; ++i) {
            if (hipEventCreate(&a[i]) != hipSuccess || hipEventCreate(&b[i]) != hipSuccess)
                return false;
        }
        ready = true;
        reset();
        return true;
    }
    void reset() {
        for (int k = 0; k < KC_COUNT; ++k) { ms[k] = 0.0; launches[k] = 0; }
    }
    void begin(int k, hipStream_t st) {
        open = false;
        if (!on || !((mask >> k) & 1u) || n >= CAP) return;
        cls[n] = k;
        (void)hipEventRecord(a[n], st);
        open = true;
    }
    // events for a launch that records them itself (hipExtLaunchKernel): the
    // interval then spans the kernel's execution, without its dispatch
    void ext(int k, hipEvent_t* e0, hipEvent_t* e1) {
        *e0 = *e1 = nullptr;
        open = false;
        if (!on || !((mask >> k) & 1u) || n >= CAP) return;
        cls[n] = k;
        *e0 = a[n];
        *e1 = b[n];
        ++n;
    }
    void end(hipStream_t st) {
        if (!open) return;
        (void)hipEventRecord(b[n], st);
        ++n;
        open = false;
    }
    // after the stream has been synchronised
    void collect() {
        for (int i = 0; i < n; ++i) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, a[i], b[i]) == hipSuccess) {
                ms[cls[i]] += t;
                launches[cls[i]] += 1;
            }
        }
        n = 0;
    }
    void destroy() {
        if (!ready) return;
        for (int i = 0; i < CAP; ++i) { (void)hipEventDestroy(a[i]); (void)hipEventDestroy(b[i]); }
        ready = false;
    }
};

inline void tbeg(Timer* t, int k, hipStream_t st) { if (t) t->begin(k, st); }
inline void tend(Timer* t, hipStream_t st) { if (t) t->end(st); }

// ---------------------------------------------------------------------------
// Instance mapping of the 2D kernels.  One launch of a kernel class covers
// every instance of a batch (a single grid is a batch of one): the device
// array g holds the instances in schedule order and start[p] is the first
// block of the instance in slot p (start[n] = the launch's block count).
// ---------------------------------------------------------------------------
enum { KB_GHOST = 0, KB_RECON, KB_RBAR, KB_GRAD, KB_FLUX0, KB_FLUX1, KB_CELLS,
       KB_FLUXUP, KB_RGRAD, KB_COUNT };

struct Batch {
    const Grid2* g;
    const int* start;
    int n;
    int xcd;          // 1: XCD-aware order of the launch's blocks
    int rev;          // 1: each XCD (or the launch) takes its range of blocks last first
};

// Work per block of the tunable kernels (cells, cells, faces).
struct Tiles {
    int recon = 32;   // 16 or 32
    int grad = 32;    // 32 or 64; 0: weak moments formed in the gradient kernel
                      // (tiles of 16 x 4 cells)
    int flux = 0;     // 64 or 128; 0: face fluxes formed inside the update kernel
    int xcd = 1;      // 1: each XCD takes a contiguous range of a launch's blocks
};

struct BatchL {
    const Grid2* dg = nullptr;     // device, n instances in schedule order
    const int* dstart = nullptr;   // device, KB_COUNT x (n + 1)
    const int* hstart = nullptr;   // host copy of dstart
    int n = 0;
    Tiles tiles;
    bool var_mu = true;            // some instance has a temperature-dependent mu
    bool dr = false;               // HWENO-DR gradients (every instance of the launch)
    bool full_grad = false;        // face gradients stored as all six (the reverse mode
                                   // reads them); else as the three combinations the
                                   // face fluxes use
    // bit k: kernel class k runs its blocks last first.  The weak-moment and
    // face-flux kernels run in the opposite order of the kernel that wrote
    // most of their input just before them (reconstruction, gradients), so
    // their first blocks read what is still in L2 and the memory-side cache;
    // the next stage's reconstruction then again runs opposite to them.
    unsigned rev = (1u << KB_RBAR) | (1u << KB_FLUX0) | (1u << KB_FLUX1) | (1u << KB_FLUXUP) |
                   (1u << KB_RGRAD);
    Batch arg(int k) const {
        return Batch{dg, dstart + k * (n + 1), n, tiles.xcd, (int)((rev >> k) & 1u)};
    }
    unsigned blocks(int k) const { return (unsigned)hstart[k * (n + 1) + n]; }
};

// Block prefix tables of every kernel class for the instances hg[0..n) (in
// schedule order) and the given tiles; out has KB_COUNT x (n + 1) entries.
void batch_blocks(const Grid2* hg, int n, const Tiles& t, int* out);

// Launchers (stream-ordered, no synchronisation).  Return hipError_t.
hipError_t launch_reset(Reduce* red, hipStream_t st);
hipError_t launch_copy_in2(const Grid2& g, const double* U, double* S, hipStream_t st);
hipError_t launch_copy_out2(const Grid2& g, const double* S, double* U, hipStream_t st);
// 2D pipeline over every instance of b; state buffers by index into Grid2::S
hipError_t launch_ghost2(const BatchL& b, int si, hipStream_t st, Timer* tm, int stage = -1);
// Mirror fill of the solid cells next to the fluid of a single masked grid
// (before the box halo); `g` is the device descriptor, n its nsolid.
hipError_t launch_solid2(const Grid2* g, int n, int si, hipStream_t st);
hipError_t launch_residual2(const BatchL& b, int si, hipStream_t st, Timer* tm);
// stage 0: write R (12) and Vhat (8) in interior layout (single grid);
// stage 1..3: RK update S[iout] from S[i0] (U^n) and S[iin] (stage input);
// src (single grid, may be null): source moments added to the residual
hipError_t launch_update2(const BatchL& b, int stage, int i0, int iin, int iout, double* R,
                          double* Vhat, hipStream_t st, Timer* tm,
                          const double* src = nullptr);
hipError_t launch_check2(const BatchL& b, int si, hipStream_t st);
hipError_t launch_reset2(const BatchL& b, hipStream_t st);
// per-instance step size from its InstState rule, halved per pending restart
hipError_t launch_dt2(const BatchL& b, hipStream_t st);
// accept (S[1] -> S[0], time, counters) or reject (halve) every active instance
hipError_t launch_commit2(const BatchL& b, hipStream_t st);
hipError_t launch_dt(Reduce* red, double cfl_h, double visc_dt, double t_left, hipStream_t st);
hipError_t launch_set_dt(Reduce* red, double dt, hipStream_t st);

hipError_t launch_copy_in1(const Grid1& g, const double* U, double* S, hipStream_t st);
hipError_t launch_copy_out1(const Grid1& g, const double* S, double* U, hipStream_t st);
hipError_t launch_ghost1(const Grid1& g, double* S, hipStream_t st, Timer* tm);
hipError_t launch_residual1(const Grid1& g, const double* S, hipStream_t st, Timer* tm);
hipError_t launch_update1(const Grid1& g, int stage, const double* S0, const double* Sin,
                          double* Sout, double* R, double* Vhat, hipStream_t st, Timer* tm,
                          const double* src = nullptr);
hipError_t launch_check1(const Grid1& g, const double* S, hipStream_t st);

// Library-owned device scratch of the allocation-free residual entry point:
// one file-scope array per device (its size is fixed at build time and it
// lives until the process ends).  static_scratch returns its device address
// on the current device, looked up once per device.
constexpr size_t STATIC_SCRATCH_BYTES = size_t(256) << 20;
hipError_t static_scratch(void** ptr);

}  // namespace hw

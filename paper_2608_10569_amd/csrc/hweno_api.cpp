// Host side of libhweno.so: context, workspace carving, the SSP-RK3 driver
// with the time-step rule and stage restart (Sec. 5 preamble of
// arXiv 2608.10569), and the C ABI of include/hweno.h.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <utility>

#include "../../include/hweno.h"
#include "hweno_kernels.h"
#include "hweno_vjp.h"

struct hweno_ctx {
    hweno_grid grid;
    hweno_physics phys;
    hweno_bcs bcs;
    hweno_options opt;
    hipStream_t stream = nullptr;
    int device = 0;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    double* S[3] = {nullptr, nullptr, nullptr};   // ghosted states; S[0] = current
    hw::Grid2 g2{};
    hw::Grid1 g1{};
    hw::Reduce* red = nullptr;
    hw::AdjWs adj{};
    double* mu_dev = nullptr;
    double* S3 = nullptr;       // 2D adjoint: fourth ghosted state (RK-step recomputation)
    double* X1 = nullptr;       // 2D adjoint: interior stage cotangents (12 per cell)
    double* X2 = nullptr;
    double t = 0.0;
    bool has_state = false;
    hw::Timer timer;
    hw::Timer* tm() { return timer.on ? &timer : nullptr; }
};

namespace {

constexpr int HALO = 4;
constexpr size_t ALIGN = 256;

size_t up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

hw::Consts make_consts(const hweno_ctx* c) {
    hw::Consts K{};
    K.gamma = c->phys.gamma;
    K.gm1 = c->phys.gamma - 1.0;
    K.Pr = c->phys.Pr;
    K.mu_ref = c->phys.mu_ref;
    K.mu_exp = c->phys.mu_exp;
    K.T_ref = c->phys.T_ref;
    K.eps_pp = c->opt.eps_pp;
    K.eps_weno = c->opt.eps_weno;
    K.linear = c->opt.linear_weights ? 1 : 0;
    K.dx = (c->grid.x1 - c->grid.x0) / c->grid.nx;
    K.idx = 1.0 / K.dx;
    if (c->grid.dim == 2) {
        K.dy = (c->grid.y1 - c->grid.y0) / c->grid.ny;
        K.idy = 1.0 / K.dy;
    } else {
        K.dy = K.dx;
        K.idy = K.idx;
    }
    return K;
}

// Wall parities (Remark 4.1): multiplier per (moment, component).
void make_side(const hweno_ctx* c, int s, hw::Side& sd) {
    const int dim = c->grid.dim;
    const int ncomp = dim + 2;
    const int axis = s / 2;               // 0: x-wall, 1: y-wall
    sd.kind = c->bcs.kind[s];
    for (int q = 0; q < 12; ++q) sd.sign[q] = 1.0;
    if (sd.kind == HWENO_BC_SLIP || sd.kind == HWENO_BC_NOSLIP) {
        for (int m = 0; m <= dim; ++m) {
            for (int comp = 0; comp < ncomp; ++comp) {
                double par = 1.0;
                const bool vel = comp >= 1 && comp <= dim;
                if (vel) {
                    const int vdir = comp - 1;   // 0: u, 1: v
                    if (sd.kind == HWENO_BC_NOSLIP || vdir == axis) par = -1.0;
                }
                const double mom = (m == 1 + axis) ? -1.0 : 1.0;   // normal moment flips
                sd.sign[m * ncomp + comp] = par * mom;
            }
        }
    }
    // inflow: primitive -> conservative
    const double* pr = c->bcs.inflow[s];
    const double g = c->phys.gamma;
    for (int q = 0; q < 4; ++q) sd.inflow[q] = 0.0;
    if (dim == 1) {
        const double r = pr[0], u = pr[1], p = pr[2];
        sd.inflow[0] = r;
        sd.inflow[1] = r * u;
        sd.inflow[2] = p / (g - 1.0) + 0.5 * r * u * u;
    } else {
        const double r = pr[0], u = pr[1], v = pr[2], p = pr[3];
        sd.inflow[0] = r;
        sd.inflow[1] = r * u;
        sd.inflow[2] = r * v;
        sd.inflow[3] = p / (g - 1.0) + 0.5 * r * (u * u + v * v);
    }
}

// Carves the workspace into the grid's arrays (or just sizes it if base == nullptr).
size_t layout(hweno_ctx* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t ndouble) -> double* {
        double* p = base ? reinterpret_cast<double*>(base + off) : nullptr;
        off += up(ndouble * sizeof(double));
        return p;
    };
    if (c->grid.dim == 2) {
        hw::Grid2& g = c->g2;
        g.nx = c->grid.nx;
        g.ny = c->grid.ny;
        g.NX = g.nx + 2 * HALO;
        g.NY = g.ny + 2 * HALO;
        g.ncell = (long long)g.NX * g.NY;
        const size_t n = (size_t)g.ncell;
        for (int k = 0; k < 3; ++k) c->S[k] = take(12 * n);
        g.xf = take(24 * n);
        g.yf = take(24 * n);
        g.xv = take(36 * n);
        g.yv = take(36 * n);
        g.wb = take(6 * n);
        g.vk = take(8 * n);
        g.vn = take(8 * n);
        g.rb = take(18 * n);
        g.gf = take(72 * n);
        g.vf = take(8 * n);
        g.fx = take(12 * n);
        g.fy = take(12 * n);
    } else {
        hw::Grid1& g = c->g1;
        g.nx = c->grid.nx;
        g.NX = g.nx + 2 * HALO;
        const size_t n = (size_t)g.NX;
        for (int k = 0; k < 3; ++k) c->S[k] = take(6 * n);
        g.pts = take(12 * n);
        g.wb = take(2 * n);
        g.vk = take(3 * n);
        g.vn = take(3 * n);
        g.rb = take(4 * n);
        g.gr = take(8 * n);
        g.fh = take(3 * n);
        g.vf = take(3 * n);
    }
    if (c->grid.dim == 2) {
        // reverse-mode workspace (zero-filled at the start of every adjoint call)
        const size_t n = (size_t)c->g2.ncell;
        hw::AdjWs& A = c->adj;
        const size_t first = off;
        A.xfb = take(24 * n);
        A.yfb = take(24 * n);
        A.xvb = take(36 * n);
        A.yvb = take(36 * n);
        A.gfb = take(72 * n);
        A.rbc = take(102 * n);
        A.rbb = take(18 * n);
        A.uc = take(136 * n);
        A.ubb = take(12 * n);
        A.base = A.xfb;
        A.count = (long long)((off - first) / sizeof(double));
        A.mupart = take((size_t)hw::adj_mu_partials2(c->g2));
        c->mu_dev = take(1);
        const size_t nint = (size_t)c->g2.nx * c->g2.ny;
        c->S3 = take(12 * n);
        c->X1 = take(12 * nint);
        c->X2 = take(12 * nint);
    }
    c->red = base ? reinterpret_cast<hw::Reduce*>(base + off) : nullptr;
    off += up(sizeof(hw::Reduce));
    c->g2.red = c->red;
    c->g1.red = c->red;
    return off;
}

hweno_status dev(hipError_t e) { return e == hipSuccess ? HWENO_OK : HWENO_E_DEVICE; }

#define TRY(x)                                   \
    do {                                         \
        hweno_status s_ = (x);                   \
        if (s_ != HWENO_OK) return s_;           \
    } while (0)

hweno_status ghost(hweno_ctx* c, double* S) {
    if (c->grid.dim == 2) return dev(hw::launch_ghost2(c->g2, S, c->stream, c->tm()));
    return dev(hw::launch_ghost1(c->g1, S, c->stream, c->tm()));
}

hweno_status residual(hweno_ctx* c, const double* S) {
    if (c->grid.dim == 2) return dev(hw::launch_residual2(c->g2, S, c->stream, c->tm()));
    return dev(hw::launch_residual1(c->g1, S, c->stream, c->tm()));
}

hweno_status update(hweno_ctx* c, int stage, const double* S0, const double* Sin, double* Sout,
                    double* R, double* V) {
    if (c->grid.dim == 2)
        return dev(hw::launch_update2(c->g2, stage, S0, Sin, Sout, R, V, c->stream, c->tm()));
    return dev(hw::launch_update1(c->g1, stage, S0, Sin, Sout, R, V, c->stream, c->tm()));
}

hweno_status read_reduce(hweno_ctx* c, hw::Reduce* r) {
    TRY(dev(hipMemcpyAsync(r, c->red, sizeof(hw::Reduce), hipMemcpyDeviceToHost, c->stream)));
    TRY(dev(hipStreamSynchronize(c->stream)));
    if (c->timer.on) c->timer.collect();
    return HWENO_OK;
}

void fill_diag(const hweno_ctx* c, const hw::Reduce& r, hweno_diag* d, int restarts,
               bool stage1_alpha) {
    if (!d) return;
    d->t = c->t;
    d->dt = r.dt;
    d->alpha_star = hw::dkey_inv(stage1_alpha ? r.alpha1_key : r.alpha_key);
    d->beta_max = hw::dkey_inv(r.beta_key);
    d->min_rho = hw::dkey_inv(r.min_rho_key);
    d->min_p = hw::dkey_inv(r.min_p_key);
    d->pp_cells = r.pp_cells;
    d->restarts = restarts;
    d->pad = 0;
}

bool valid_kind(int k) { return k >= HWENO_BC_PERIODIC && k <= HWENO_BC_NOSLIP; }

}  // namespace

extern "C" {

HWENO_API hweno_status hweno_default_options(hweno_options* o) {
    if (!o) return HWENO_E_INVAL;
    o->cfl = 0.6;
    o->b_visc = 0.001;
    o->eps_pp = 1e-12;
    o->eps_weno = 1e-8;
    o->t_final = 0.0;
    o->linear_weights = 0;
    o->max_halvings = 40;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_create(const hweno_grid* grid, const hweno_physics* phys,
                                    const hweno_bcs* bcs, const hweno_options* opt,
                                    hweno_ctx** out) {
    if (!grid || !phys || !bcs || !opt || !out) return HWENO_E_INVAL;
    *out = nullptr;
    if (grid->dim != 1 && grid->dim != 2) return HWENO_E_INVAL;
    if (grid->nx < 4 || !(grid->x1 > grid->x0)) return HWENO_E_INVAL;
    if (grid->dim == 2 && (grid->ny < 4 || !(grid->y1 > grid->y0))) return HWENO_E_INVAL;
    if (!(phys->gamma > 1.0) || !(phys->Pr > 0.0) || !(phys->mu_ref >= 0.0) ||
        !(phys->T_ref > 0.0) || !std::isfinite(phys->mu_exp))
        return HWENO_E_INVAL;
    if (!(opt->cfl > 0.0) || !(opt->eps_pp > 0.0) || !(opt->eps_weno > 0.0) ||
        opt->max_halvings < 0)
        return HWENO_E_INVAL;
    const int nsides = 2 * grid->dim;
    for (int s = 0; s < nsides; ++s) {
        if (!valid_kind(bcs->kind[s])) return HWENO_E_INVAL;
        if (bcs->kind[s] == HWENO_BC_INFLOW) {
            const double r = bcs->inflow[s][0];
            const double p = bcs->inflow[s][grid->dim == 1 ? 2 : 3];
            if (!(r > 0.0) || !(p > 0.0)) return HWENO_E_INVAL;
        }
    }
    for (int a = 0; a < grid->dim; ++a) {
        const bool p0 = bcs->kind[2 * a] == HWENO_BC_PERIODIC;
        const bool p1 = bcs->kind[2 * a + 1] == HWENO_BC_PERIODIC;
        if (p0 != p1) return HWENO_E_INVAL;
    }
    hweno_ctx* c = new (std::nothrow) hweno_ctx;
    if (!c) return HWENO_E_INVAL;
    c->grid = *grid;
    c->phys = *phys;
    c->bcs = *bcs;
    c->opt = *opt;
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    c->ws_bytes = layout(c, nullptr);
    const hw::Consts K = make_consts(c);
    c->g2.K = K;
    c->g1.K = K;
    for (int s = 0; s < 4; ++s) make_side(c, s, c->g2.side[s]);
    for (int s = 0; s < 2; ++s) make_side(c, s, c->g1.side[s]);
    *out = c;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_destroy(hweno_ctx* c) {
    if (!c) return HWENO_E_INVAL;
    c->timer.destroy();
    delete c;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_workspace_bytes(const hweno_ctx* c, size_t* bytes) {
    if (!c || !bytes) return HWENO_E_INVAL;
    *bytes = c->ws_bytes;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_set_workspace(hweno_ctx* c, void* p, size_t bytes) {
    if (!c || !p) return HWENO_E_INVAL;
    if (bytes < c->ws_bytes || (reinterpret_cast<uintptr_t>(p) % ALIGN) != 0)
        return HWENO_E_WORKSPACE;
    c->ws = static_cast<char*>(p);
    layout(c, c->ws);
    c->has_state = false;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_set_stream(hweno_ctx* c, void* s) {
    if (!c) return HWENO_E_INVAL;
    c->stream = static_cast<hipStream_t>(s);
    return HWENO_OK;
}

HWENO_API hweno_status hweno_set_state(hweno_ctx* c, const double* U, double t) {
    if (!c || !U || !std::isfinite(t)) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->grid.dim == 2) TRY(dev(hw::launch_copy_in2(c->g2, U, c->S[0], c->stream)));
    else TRY(dev(hw::launch_copy_in1(c->g1, U, c->S[0], c->stream)));
    c->t = t;
    c->has_state = true;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_get_state(hweno_ctx* c, double* U, double* t) {
    if (!c || !U) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    if (c->grid.dim == 2) TRY(dev(hw::launch_copy_out2(c->g2, c->S[0], U, c->stream)));
    else TRY(dev(hw::launch_copy_out1(c->g1, c->S[0], U, c->stream)));
    if (t) *t = c->t;
    return HWENO_OK;
}

HWENO_API hweno_status hweno_residual(hweno_ctx* c, const double* U, double* R, double* V,
                                      hweno_diag* diag) {
    if (!c || !U || !R || !V) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    double* S = c->S[2];
    if (c->grid.dim == 2) TRY(dev(hw::launch_copy_in2(c->g2, U, S, c->stream)));
    else TRY(dev(hw::launch_copy_in1(c->g1, U, S, c->stream)));
    TRY(dev(hw::launch_reset(c->red, c->stream)));
    TRY(ghost(c, S));
    TRY(residual(c, S));
    TRY(update(c, 0, S, S, S, R, V));
    if (diag) {
        hw::Reduce r;
        TRY(read_reduce(c, &r));
        fill_diag(c, r, diag, 0, false);
        diag->dt = 0.0;
        diag->min_rho = diag->min_p = NAN;
    }
    return HWENO_OK;
}

HWENO_API hweno_status hweno_rk_step(hweno_ctx* c, double dt, hweno_diag* diag) {
    if (!c || std::isnan(dt)) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    const bool auto_dt = !(dt > 0.0);
    const double h = c->grid.dim == 2 ? std::fmin(c->g2.K.dx, c->g2.K.dy) : c->g1.K.dx;
    double visc = INFINITY;
    if (c->opt.b_visc > 0.0 && c->phys.mu_ref > 0.0) visc = c->opt.b_visc * h * h / c->phys.mu_ref;
    const double t_left = c->opt.t_final > 0.0 ? c->opt.t_final - c->t : INFINITY;
    if (auto_dt && !(t_left > 0.0)) {   // already at t_final: nothing to do
        if (diag) {
            std::memset(diag, 0, sizeof(*diag));
            diag->t = c->t;
        }
        return HWENO_OK;
    }
    double cur = dt;
    int restarts = 0;
    hw::Reduce r;
    for (;;) {
        double* S0 = c->S[0];
        double* S1 = c->S[1];
        double* S2 = c->S[2];
        TRY(dev(hw::launch_reset(c->red, c->stream)));
        if (restarts == 0) {
            if (c->grid.dim == 2) TRY(dev(hw::launch_check2(c->g2, S0, c->stream)));
            else TRY(dev(hw::launch_check1(c->g1, S0, c->stream)));
        }
        TRY(ghost(c, S0));
        TRY(residual(c, S0));
        if (auto_dt && restarts == 0)
            TRY(dev(hw::launch_dt(c->red, c->opt.cfl * h, visc, t_left, c->stream)));
        else
            TRY(dev(hw::launch_set_dt(c->red, cur, c->stream)));
        TRY(update(c, 1, S0, S0, S1, nullptr, nullptr));
        TRY(ghost(c, S1));
        TRY(residual(c, S1));
        TRY(update(c, 2, S0, S1, S2, nullptr, nullptr));
        TRY(ghost(c, S2));
        TRY(residual(c, S2));
        TRY(update(c, 3, S0, S2, S1, nullptr, nullptr));
        TRY(read_reduce(c, &r));
        if (restarts == 0 && r.bad[0] != 0) return HWENO_E_NONFINITE;
        if (!(r.dt > 0.0) || !std::isfinite(r.dt)) return HWENO_E_NONFINITE;
        if (r.bad[1] == 0 && r.bad[2] == 0 && r.bad[3] == 0) break;
        if (restarts >= c->opt.max_halvings) return HWENO_E_INADMISSIBLE;
        ++restarts;
        cur = 0.5 * r.dt;
    }
    std::swap(c->S[0], c->S[1]);
    c->t += r.dt;
    fill_diag(c, r, diag, restarts, true);
    return HWENO_OK;
}

HWENO_API hweno_status hweno_residual_vjp(hweno_ctx* c, const double* U, const double* Rbar,
                                          const double* Vbar, double* Ubar, double* mu_bar) {
    if (!c || !U || !Rbar || !Ubar) return HWENO_E_INVAL;
    if (c->grid.dim != 2 || c->phys.mu_exp != 0.0) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    double* S = c->S[2];
    TRY(dev(hw::launch_copy_in2(c->g2, U, S, c->stream)));
    TRY(dev(hw::launch_reset(c->red, c->stream)));
    TRY(ghost(c, S));
    TRY(residual(c, S));
    hw::AdjIn A{Rbar, Vbar, 1.0, 1.0};
    TRY(dev(hw::launch_vjp2(c->g2, A, c->adj, S, Ubar, c->mu_dev, 0, c->stream)));
    if (mu_bar) {
        TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                               c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
    }
    return HWENO_OK;
}

// Reverse mode of one SSP-RK3 step with the step size frozen (eq. (2.12)):
//   U1 = B(U0) + dt F(U0),  U2 = 3/4 B(U0) + 1/4 (B(U1) + dt F(U1)),
//   U3 = 1/3 B(U0) + 2/3 (B(U2) + dt F(U2)),   B(U) = (ubar, hat-v(U)).
// The stages are recomputed from U0 with the forward kernels, then the three
// residual adjoints run in reverse with the stage cotangents as seeds.
HWENO_API hweno_status hweno_rk_step_vjp(hweno_ctx* c, const double* U0, double dt,
                                         const double* U3bar, double* U0bar, double* mu_bar) {
    if (!c || !U0 || !U3bar || !U0bar || !(dt > 0.0) || !std::isfinite(dt)) return HWENO_E_INVAL;
    if (c->grid.dim != 2 || c->phys.mu_exp != 0.0) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    const hw::Grid2& g = c->g2;
    const long long nint = (long long)g.nx * g.ny;
    double* Sa = c->S[1];   // U0
    double* Sb = c->S[2];   // U1
    double* Sc = c->S3;     // U2
    // forward recomputation of the two intermediate stages
    TRY(dev(hw::launch_copy_in2(g, U0, Sa, c->stream)));
    TRY(dev(hw::launch_reset(c->red, c->stream)));
    TRY(dev(hw::launch_set_dt(c->red, dt, c->stream)));
    TRY(ghost(c, Sa));
    TRY(residual(c, Sa));
    TRY(update(c, 1, Sa, Sa, Sb, nullptr, nullptr));
    TRY(ghost(c, Sb));
    TRY(residual(c, Sb));
    TRY(update(c, 2, Sa, Sb, Sc, nullptr, nullptr));
    auto vjp_at = [&](double* S, const double* Rb, double rs, double vs, double* out, int acc) {
        TRY(dev(hw::launch_reset(c->red, c->stream)));
        TRY(ghost(c, S));
        TRY(residual(c, S));
        hw::AdjIn A{Rb, Rb + 4 * nint, rs, vs};
        return dev(hw::launch_vjp2(g, A, c->adj, S, out, c->mu_dev, acc, c->stream));
    };
    // stage 3: seeds 2/3 dt U3bar (residual) and 2/3 U3bar (modified moments)
    TRY(vjp_at(Sc, U3bar, (2.0 / 3.0) * dt, 2.0 / 3.0, c->X2, 0));
    TRY(dev(hw::launch_axpy(c->X2, U3bar, 2.0 / 3.0, 4 * nint, c->stream)));      // U2bar
    // stage 2: seeds 1/4 dt U2bar and 1/4 U2bar
    TRY(vjp_at(Sb, c->X2, 0.25 * dt, 0.25, c->X1, 1));
    TRY(dev(hw::launch_axpy(c->X1, c->X2, 0.25, 4 * nint, c->stream)));           // U1bar
    // B(U0)-bar = 1/3 U3bar + 3/4 U2bar + U1bar (into X2)
    TRY(dev(hw::launch_lin3(c->X2, U3bar, 1.0 / 3.0, 0.75, c->X1, 12 * nint, c->stream)));
    // stage 1: residual seed dt U1bar, modified-moment seed B(U0)-bar
    TRY(dev(hw::launch_reset(c->red, c->stream)));
    TRY(ghost(c, Sa));
    TRY(residual(c, Sa));
    {
        hw::AdjIn A{c->X1, c->X2 + 4 * nint, dt, 1.0};
        TRY(dev(hw::launch_vjp2(g, A, c->adj, Sa, U0bar, c->mu_dev, 1, c->stream)));
    }
    TRY(dev(hw::launch_axpy(U0bar, c->X2, 1.0, 4 * nint, c->stream)));
    if (mu_bar) {
        TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                               c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
    }
    return HWENO_OK;
}

HWENO_API hweno_status hweno_set_timing(hweno_ctx* c, int enable) {
    if (!c) return HWENO_E_INVAL;
    if (enable) {
        if (!c->timer.init()) return HWENO_E_DEVICE;
        c->timer.on = true;
    } else {
        c->timer.on = false;
    }
    return HWENO_OK;
}

HWENO_API hweno_status hweno_get_timing(hweno_ctx* c, hweno_timing* out, int reset) {
    if (!c || !out) return HWENO_E_INVAL;
    if (c->timer.ready) {
        TRY(dev(hipStreamSynchronize(c->stream)));
        c->timer.collect();
    }
    for (int k = 0; k < 8; ++k) {
        out->ms[k] = c->timer.ready ? c->timer.ms[k] : 0.0;
        out->launches[k] = c->timer.ready ? c->timer.launches[k] : 0;
    }
    if (reset && c->timer.ready) c->timer.reset();
    return HWENO_OK;
}

HWENO_API const char* hweno_status_string(hweno_status s) {
    switch (s) {
        case HWENO_OK: return "ok";
        case HWENO_E_INVAL: return "invalid argument";
        case HWENO_E_DEVICE: return "HIP device error";
        case HWENO_E_WORKSPACE: return "workspace missing, too small or misaligned";
        case HWENO_E_INADMISSIBLE: return "stage inadmissible after the maximum number of halvings";
        case HWENO_E_NONFINITE: return "state not finite or not positive";
        case HWENO_E_STATE: return "no state set";
    }
    return "unknown status";
}

}  // extern "C"

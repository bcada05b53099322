// Host side of libhweno.so: contexts (one grid, or a batch of 2D grids),
// workspace carving, the SSP-RK3 driver with the time-step rule and stage
// restart (Sec. 5 preamble of arXiv 2608.10569), the graph-captured batched
// run, the tile autotuner, and the C ABI of include/hweno.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <utility>
#include <vector>

#include "../../include/hweno.h"
#include "hweno_kernels.h"
#include "hweno_vjp.h"

namespace {

// One grid's problem statement.
struct Inst {
    hweno_grid grid;
    hweno_physics phys;
    hweno_bcs bcs;
    hweno_options opt;
};

}  // namespace

struct hweno_ctx {
    bool batch = false;
    std::vector<Inst> in;              // instances (one for a single grid)
    hipStream_t stream = nullptr;
    int device = 0;
    size_t ws_bytes = 0;
    char* ws = nullptr;
    // 2D: host copies of every instance's grid (by instance id), their device
    // copies in schedule order, the block tables and the per-instance state
    std::vector<hw::Grid2> hg;
    std::vector<int> order;            // slot -> instance id
    hw::Grid2* dg = nullptr;
    int* dstart = nullptr;
    std::vector<int> hstart;
    // batches of two or more instances: two groups of consecutive slots with
    // about equal cells, recorded as two concurrent chains of the run's graph
    // (one group's reconstruction beside the other's memory-bound kernels)
    int ngroups = 1;
    int* dstart_g[2] = {nullptr, nullptr};
    std::vector<int> hstart_g[2];
    hw::BatchL blg[2];
    hw::Tiles tiles;
    int order_mode = 0;                // 0: as given, 1: largest first
    hw::BatchL bl;
    hw::InstState* dst = nullptr;      // device, by instance id
    std::vector<hw::InstState> hst;    // host copy
    hw::Reduce* red = nullptr;         // device, by instance id
    int cur = 0;                       // single 2D grid: current state is hg[0].S[cur]
    // 1D
    // ghosted states; S1[0] = current, 1 and 2 the step's stages, 3 and 4
    // the reverse mode's recomputed stages
    double* S1[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};
    hw::Grid1 g1{};
    // reverse mode (single 2D grid; 1D grid)
    hw::AdjWs adj{};
    hw::AdjWs1 adj1{};
    // keep_stages (single 2D grid): residual intermediates of RK stages 2 and 3
    // in arrays of their own, described by stage[k] (host) / dstage + k
    // (device) and launched through blstage[k]
    hw::Grid2 stage[2]{};
    hw::Grid2* dstage = nullptr;
    hw::BatchL blstage[2];
    double* mu_dev = nullptr;
    double* X1 = nullptr;              // interior stage cotangents (12 per cell)
    double* X2 = nullptr;
    // recorded steps (single 2D grid, caller's buffer): per slot the three
    // stage inputs and their residual intermediates, described by rec_desc
    // (host) / rec_ddesc (device, 3 per slot); rec_dt > 0 once recorded
    char* rec_base = nullptr;
    int rec_slots = 0;
    std::vector<hw::Grid2> rec_desc;
    hw::Grid2* rec_ddesc = nullptr;
    std::vector<double> rec_dt;
    double t = 0.0;
    bool has_state = false;
    bool state_checked = false;        // the current state passed the admissibility check
    std::vector<char> have;            // batch: state set, per instance
    // batched run: graphs of `gsteps` steps and of one step
    hipGraphExec_t gexec = nullptr;
    int gsteps = 0;
    hipGraphExec_t gexec1 = nullptr;
    hipStream_t cap_stream = nullptr;  // private stream the graphs are recorded on
    hipStream_t cap_stream2 = nullptr; // the second group's chain while recording
    hw::Timer timer;
    // single 2D grid: inflow profiles (conservative, 4 per boundary cell) and
    // their workspace copies
    std::vector<double> prof_host[4];
    double* prof_dev[4] = {nullptr, nullptr, nullptr, nullptr};
    // inflow profiles of the three stages of the next fixed-step call, per side
    std::vector<double> stage_host[4];
    double* stage_dev[4] = {nullptr, nullptr, nullptr, nullptr};
    // masked domain (single 2D grid): interior mask and the mirror list
    std::vector<unsigned char> solid_host;
    std::vector<int> sdst_host, ssrc_host, sdir_host;
    int solid_wall = 0;
    // solid cells that hold a prescribed state (hweno_set_solid_state)
    std::vector<unsigned char> fixed_host;
    double fixed_cons[4] = {0.0, 0.0, 0.0, 0.0};
    unsigned char* solid_dev = nullptr;
    int* sdst_dev = nullptr;
    int* ssrc_dev = nullptr;
    int* sdir_dev = nullptr;
    // the mirror list grouped by source, for the reverse mode (AdjWs::ssrcu ..)
    int* ssrcu_dev = nullptr;
    int* sstart_dev = nullptr;
    int* sord_dev = nullptr;
    // allocation-free residual (hweno_residual_noalloc): the descriptors it
    // copies into the library's static scratch, kept here so that the copies
    // read host memory that outlives the call
    hw::Grid2 sgrid{};
    hw::InstState sstate{};
    int sstart[2 * hw::KB_COUNT] = {};
    hw::Timer* tm() { return timer.on ? &timer : nullptr; }
    const Inst& i0() const { return in[0]; }
    int dim() const { return in[0].grid.dim; }
};

namespace {

constexpr int HALO = 4;
constexpr size_t ALIGN = 256;

size_t up(size_t n) { return (n + ALIGN - 1) / ALIGN * ALIGN; }

hw::Consts make_consts(const Inst& c) {
    hw::Consts K{};
    K.gamma = c.phys.gamma;
    K.gm1 = c.phys.gamma - 1.0;
    K.igm1 = 1.0 / K.gm1;
    K.gPr = c.phys.gamma / c.phys.Pr;
    K.Pr = c.phys.Pr;
    K.mu_ref = c.phys.mu_ref;
    K.mu_exp = c.phys.mu_exp;
    K.T_ref = c.phys.T_ref;
    K.eps_pp = c.opt.eps_pp;
    K.eps_weno = c.opt.eps_weno;
    K.linear = c.opt.linear_weights ? 1 : 0;
    K.linear_grad = c.opt.linear_gradients ? 1 : 0;
    K.dr = c.opt.gradients ? 1 : 0;
    K.dx = (c.grid.x1 - c.grid.x0) / c.grid.nx;
    K.idx = 1.0 / K.dx;
    if (c.grid.dim == 2) {
        K.dy = (c.grid.y1 - c.grid.y0) / c.grid.ny;
        K.idy = 1.0 / K.dy;
    } else {
        K.dy = K.dx;
        K.idy = K.idx;
    }
    return K;
}

// Wall parities (Remark 4.1): multiplier per (moment, component).
void make_side(const Inst& c, int s, hw::Side& sd) {
    const int dim = c.grid.dim;
    const int ncomp = dim + 2;
    const int axis = s / 2;               // 0: x-wall, 1: y-wall
    sd.kind = c.bcs.kind[s];
    sd.prof = nullptr;
    sd.prof_stage = nullptr;
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
    const double* pr = c.bcs.inflow[s];
    const double g = c.phys.gamma;
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

// Step-rule constants of an instance (Sec. 5 preamble).
void rule(const Inst& c, double* cfl_h, double* visc_dt) {
    const double dx = (c.grid.x1 - c.grid.x0) / c.grid.nx;
    const double h = c.grid.dim == 2 ? std::fmin(dx, (c.grid.y1 - c.grid.y0) / c.grid.ny) : dx;
    *cfl_h = c.opt.cfl * h;
    *visc_dt = INFINITY;
    if (c.opt.b_visc > 0.0 && c.phys.mu_ref > 0.0) *visc_dt = c.opt.b_visc * h * h / c.phys.mu_ref;
}

// Carves the workspace into the grids' arrays (or just sizes it if base == nullptr).
size_t layout(hweno_ctx* c, char* base) {
    size_t off = 0;
    auto take = [&](size_t ndouble) -> hw::gdouble* {
        hw::gdouble* p = base ? (hw::gdouble*)(base + off) : nullptr;
        off += up(ndouble * sizeof(double));
        return p;
    };
    auto take_bytes = [&](size_t nb) -> char* {
        char* p = base ? base + off : nullptr;
        off += up(nb);
        return p;
    };
    const int n = (int)c->in.size();
    if (c->dim() == 1) {
        hw::Grid1& g = c->g1;
        g.nx = c->i0().grid.nx;
        g.NX = g.nx + 2 * HALO;
        const size_t m = (size_t)g.NX;
        for (int k = 0; k < 5; ++k) c->S1[k] = take(6 * m);
        g.pts = take(12 * m);
        g.wb = take(2 * m);
        g.vk = take(3 * m);
        g.vn = take(3 * m);
        g.rb = take(4 * m);
        g.gr = take(8 * m);
        g.fh = take(3 * m);
        g.vf = take(3 * m);
        c->red = reinterpret_cast<hw::Reduce*>(take_bytes(sizeof(hw::Reduce)));
        g.red = (HW_GLOBAL hw::Reduce*)c->red;
        // reverse-mode workspace (the first three arrays zero-filled by every
        // adjoint call, in one region)
        hw::AdjWs1& A = c->adj1;
        const size_t nm = m + (size_t)g.nx + 1;
        A.ptsb = take(12 * m + 8 * m + nm);
        A.grb = A.ptsb ? A.ptsb + 12 * m : nullptr;
        A.mupart = A.ptsb ? A.grb + 8 * m : nullptr;
        A.base = A.ptsb;
        A.count = (long long)(20 * m + nm);
        A.rbc = take(10 * m);
        A.uc = take(15 * m);
        A.ub = take(6 * m);
        c->mu_dev = take(1);
        c->X1 = take(6 * (size_t)g.nx);
        c->X2 = take(6 * (size_t)g.nx);
        return off;
    }
    for (int p = 0; p < n; ++p) {
        hw::Grid2& g = c->hg[p];
        const size_t m = (size_t)g.ncell;
        for (int k = 0; k < 3; ++k) g.S[k] = take(12 * m);
        g.S[3] = c->batch ? nullptr : take(12 * m);   // reverse-mode recomputation
        g.xf = take(24 * m);
        g.yf = take(24 * m);
        // the full volume values and the six face gradients are the reverse
        // mode's, which batches never run
        g.xv = c->batch ? nullptr : take(36 * m);
        g.yv = c->batch ? nullptr : take(36 * m);
        g.vc = take(2 * hw::VC_B * m);
        g.wb = take(6 * m);
        g.vk = take(8 * m);
        g.vn = take(8 * m);
        g.rb = take(18 * m);
        g.gf = take((c->batch ? 36 : 72) * m);
        g.vf = take(8 * m);
        g.fx = take(8 * m);
        g.fy = take(8 * m);
    }
    if (!c->batch) {
        // reverse-mode workspace: every slot an adjoint call reads is written
        // earlier in the same call (no clearing)
        const size_t m = (size_t)c->hg[0].ncell;
        hw::AdjWs& A = c->adj;
        A.xfb = take(24 * m);
        A.yfb = take(24 * m);
        A.xvb = take(36 * m);
        A.yvb = take(36 * m);
        A.gfb = take(72 * m);
        A.rbc = take(102 * m);
        A.rbb = take(18 * m);
        A.uc = take(136 * m);
        A.rcb = take(128 * m);
        A.rrb = take(32 * m);
        A.rlim = take(4 * m);
        A.ubb = take(12 * m);
        A.mupart = take((size_t)hw::adj_mu_partials2(c->hg[0]));
        c->mu_dev = take(1);
        const size_t nint = (size_t)c->hg[0].nx * c->hg[0].ny;
        c->X1 = take(12 * nint);
        c->X2 = take(12 * nint);
        A.rbm = take(12 * nint);
        A.vbm = take(8 * nint);
        for (int sd = 0; sd < 4; ++sd) {
            const size_t len = (size_t)(sd < 2 ? c->hg[0].ny : c->hg[0].nx);
            c->prof_dev[sd] = take(4 * len);
            c->stage_dev[sd] = take(12 * len);
        }
        c->solid_dev = reinterpret_cast<unsigned char*>(take_bytes(nint));
        c->sdst_dev = reinterpret_cast<int*>(take_bytes(nint * sizeof(int)));
        c->ssrc_dev = reinterpret_cast<int*>(take_bytes(nint * sizeof(int)));
        c->sdir_dev = reinterpret_cast<int*>(take_bytes(nint * sizeof(int)));
        c->ssrcu_dev = reinterpret_cast<int*>(take_bytes(nint * sizeof(int)));
        c->sstart_dev = reinterpret_cast<int*>(take_bytes((nint + 1) * sizeof(int)));
        c->sord_dev = reinterpret_cast<int*>(take_bytes(nint * sizeof(int)));
        if (c->i0().opt.keep_stages) {
            for (int k = 0; k < 2; ++k) {
                hw::Grid2& st = c->stage[k];
                st.xf = take(24 * m);
                st.yf = take(24 * m);
                st.xv = take(36 * m);
                st.yv = take(36 * m);
                st.vc = take(2 * hw::VC_B * m);
                st.wb = take(6 * m);
                st.vk = take(8 * m);
                st.rb = take(18 * m);
                st.gf = take(72 * m);
                st.vf = take(8 * m);
                st.fx = take(8 * m);
                st.fy = take(8 * m);
            }
            c->dstage = reinterpret_cast<hw::Grid2*>(take_bytes(2 * sizeof(hw::Grid2)));
        }
    }
    c->red = reinterpret_cast<hw::Reduce*>(take_bytes(n * sizeof(hw::Reduce)));
    c->dst = reinterpret_cast<hw::InstState*>(take_bytes(n * sizeof(hw::InstState)));
    c->dg = reinterpret_cast<hw::Grid2*>(take_bytes(n * sizeof(hw::Grid2)));
    c->dstart = reinterpret_cast<int*>(take_bytes(hw::KB_COUNT * (n + 1) * sizeof(int)));
    if (c->batch)
        for (int k = 0; k < 2; ++k)
            c->dstart_g[k] = reinterpret_cast<int*>(take_bytes(hw::KB_COUNT * (n + 1) * sizeof(int)));
    for (int p = 0; p < n; ++p) {
        c->hg[p].red = (HW_GLOBAL hw::Reduce*)(c->red ? c->red + p : nullptr);
        c->hg[p].st = (HW_GLOBAL hw::InstState*)(c->dst ? c->dst + p : nullptr);
    }
    return off;
}

// A failed call leaves its error pending in the runtime; it is cleared here so
// that it is reported once, by the call that caused it.
hweno_status dev(hipError_t e) {
    if (e == hipSuccess) return HWENO_OK;
    (void)hipGetLastError();
    return HWENO_E_DEVICE;
}

#define TRY(x)                                   \
    do {                                         \
        hweno_status s_ = (x);                   \
        if (s_ != HWENO_OK) return s_;           \
    } while (0)

// Every exported function runs its body inside GUARD_BEGIN / GUARD_END, so no
// C++ exception crosses the C ABI.  The only ones the host code can raise are
// the standard containers' allocation failures (std::bad_alloc,
// std::length_error), reported as HWENO_E_NOMEM; the context is left as it
// was before the call wherever the failing allocation precedes any change.
#define GUARD_BEGIN try {
#define GUARD_END                                \
    }                                            \
    catch (...) {                                \
        return HWENO_E_NOMEM;                    \
    }

void drop_graphs(hweno_ctx* c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    if (c->gexec1) (void)hipGraphExecDestroy(c->gexec1);
    c->gexec = c->gexec1 = nullptr;
    c->gsteps = 0;
}

// Carves a recording buffer into nslots slots, each the three ghosted stage
// inputs of one RK step and the full-layout intermediates of its three stage
// residuals, then the slots' device descriptors (3 per slot: the grid's own,
// with S[0..2] the slot's stage inputs, S[3] the grid's scratch state, and
// the intermediate arrays of that stage).  base == nullptr: size only.
size_t record_layout(const hweno_ctx* c, char* base, int nslots, std::vector<hw::Grid2>* desc,
                     hw::Grid2** ddesc) {
    size_t off = 0;
    auto take = [&](size_t nd) -> hw::gdouble* {
        hw::gdouble* p = base ? (hw::gdouble*)(base + off) : nullptr;
        off += up(nd * sizeof(double));
        return p;
    };
    const hw::Grid2& g = c->hg[0];
    const size_t m = (size_t)g.ncell;
    if (desc) desc->assign(3 * (size_t)nslots, g);
    for (int sl = 0; sl < nslots; ++sl) {
        hw::gdouble* S[3];
        for (int k = 0; k < 3; ++k) S[k] = take(12 * m);
        for (int k = 0; k < 3; ++k) {
            hw::Grid2 d = g;
            for (int q = 0; q < 3; ++q) d.S[q] = S[q];
            d.S[3] = g.S[3];
            d.xf = take(24 * m);
            d.yf = take(24 * m);
            d.xv = take(36 * m);
            d.yv = take(36 * m);
            d.vc = take(2 * hw::VC_B * m);
            d.wb = take(6 * m);
            d.vk = take(8 * m);
            d.rb = take(18 * m);
            d.gf = take(72 * m);
            d.vf = take(8 * m);
            d.fx = take(8 * m);
            d.fy = take(8 * m);
            if (desc) (*desc)[3 * (size_t)sl + k] = d;
        }
    }
    char* dd = base ? base + off : nullptr;
    off += up(3 * (size_t)nslots * sizeof(hw::Grid2));
    if (ddesc) *ddesc = reinterpret_cast<hw::Grid2*>(dd);
    return off;
}

hweno_status upload_record(hweno_ctx* c) {
    if (c->rec_slots <= 0) return HWENO_OK;
    record_layout(c, c->rec_base, c->rec_slots, &c->rec_desc, &c->rec_ddesc);
    TRY(dev(hipMemcpyAsync(c->rec_ddesc, c->rec_desc.data(),
                           c->rec_desc.size() * sizeof(hw::Grid2), hipMemcpyHostToDevice,
                           c->stream)));
    return dev(hipStreamSynchronize(c->stream));
}

// Schedule order, block tables and device grid array (synchronous).
hweno_status upload_grids(hweno_ctx* c) {
    const int n = (int)c->hg.size();
    c->order.resize(n);
    for (int p = 0; p < n; ++p) c->order[p] = p;
    if (c->order_mode == 1) {
        std::stable_sort(c->order.begin(), c->order.end(), [&](int a, int b) {
            return c->hg[a].ncell > c->hg[b].ncell;
        });
    }
    std::vector<hw::Grid2> slots(n);
    for (int p = 0; p < n; ++p) slots[p] = c->hg[c->order[p]];
    c->hstart.assign(hw::KB_COUNT * (n + 1), 0);
    hw::batch_blocks(slots.data(), n, c->tiles, c->hstart.data());
    TRY(dev(hipMemcpyAsync(c->dg, slots.data(), n * sizeof(hw::Grid2), hipMemcpyHostToDevice,
                           c->stream)));
    TRY(dev(hipMemcpyAsync(c->dstart, c->hstart.data(), c->hstart.size() * sizeof(int),
                           hipMemcpyHostToDevice, c->stream)));
    TRY(dev(hipStreamSynchronize(c->stream)));
    c->bl.dg = c->dg;
    c->bl.dstart = c->dstart;
    c->bl.hstart = c->hstart.data();
    c->bl.n = n;
    c->bl.tiles = c->tiles;
    c->bl.var_mu = false;
    for (const Inst& in : c->in) c->bl.var_mu = c->bl.var_mu || in.phys.mu_exp != 0.0;
    c->bl.dr = c->i0().opt.gradients != 0;   // the same for every instance (checked)
    c->ngroups = 1;
    if (c->batch && n >= 2 && c->dstart_g[0]) {
        // split the slots where the two groups' cells are closest to equal
        long long tot = 0, pre = 0;
        for (const hw::Grid2& gg : slots) tot += gg.ncell;
        int h = 1;
        long long best = -1;
        for (int k = 1; k < n; ++k) {
            pre += slots[k - 1].ncell;
            const long long d = pre * 2 > tot ? pre * 2 - tot : tot - pre * 2;
            if (best < 0 || d < best) {
                best = d;
                h = k;
            }
        }
        for (int q = 0; q < 2; ++q) {
            const int off = q ? h : 0, ng = q ? n - h : h;
            c->hstart_g[q].assign(hw::KB_COUNT * (ng + 1), 0);
            hw::batch_blocks(slots.data() + off, ng, c->tiles, c->hstart_g[q].data());
            TRY(dev(hipMemcpyAsync(c->dstart_g[q], c->hstart_g[q].data(),
                                   c->hstart_g[q].size() * sizeof(int), hipMemcpyHostToDevice,
                                   c->stream)));
            hw::BatchL& b = c->blg[q];
            b = c->bl;
            b.dg = c->dg + off;
            b.dstart = c->dstart_g[q];
            b.hstart = c->hstart_g[q].data();
            b.n = ng;
            b.var_mu = false;
            for (int k = off; k < off + ng; ++k)
                b.var_mu = b.var_mu || c->in[c->order[k]].phys.mu_exp != 0.0;
        }
        TRY(dev(hipStreamSynchronize(c->stream)));
        c->ngroups = 2;
    }
    if (!c->batch && c->dstage) {
        // descriptors of the stage intermediates: the grid's own, with the
        // intermediate arrays of set k
        hw::Grid2 d[2];
        for (int k = 0; k < 2; ++k) {
            const hw::Grid2& st = c->stage[k];
            d[k] = c->hg[0];
            d[k].xf = st.xf;
            d[k].yf = st.yf;
            d[k].xv = st.xv;
            d[k].yv = st.yv;
            d[k].vc = st.vc;
            d[k].wb = st.wb;
            d[k].vk = st.vk;
            d[k].rb = st.rb;
            d[k].gf = st.gf;
            d[k].vf = st.vf;
            d[k].fx = st.fx;
            d[k].fy = st.fy;
        }
        TRY(dev(hipMemcpyAsync(c->dstage, d, sizeof d, hipMemcpyHostToDevice, c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
        for (int k = 0; k < 2; ++k) {
            c->stage[k] = d[k];
            c->blstage[k] = c->bl;
            c->blstage[k].dg = c->dstage + k;
        }
    }
    if (!c->batch) TRY(upload_record(c));
    drop_graphs(c);
    return HWENO_OK;
}

// Inflow profiles of a single 2D grid into the workspace; the grid's sides
// point at them (or at nothing).  The grid descriptors are uploaded after.
hweno_status upload_profiles(hweno_ctx* c) {
    for (int sd = 0; sd < 4; ++sd) {
        const std::vector<double>& h = c->prof_host[sd];
        c->hg[0].side[sd].prof = nullptr;
        if (!h.empty()) {
            TRY(dev(hipMemcpyAsync(c->prof_dev[sd], h.data(), h.size() * sizeof(double),
                                   hipMemcpyHostToDevice, c->stream)));
            c->hg[0].side[sd].prof = (const hw::gdouble*)c->prof_dev[sd];
        }
        const std::vector<double>& q = c->stage_host[sd];
        c->hg[0].side[sd].prof_stage = nullptr;
        if (!q.empty()) {
            TRY(dev(hipMemcpyAsync(c->stage_dev[sd], q.data(), q.size() * sizeof(double),
                                   hipMemcpyHostToDevice, c->stream)));
            c->hg[0].side[sd].prof_stage = (const hw::gdouble*)c->stage_dev[sd];
        }
    }
    return dev(hipStreamSynchronize(c->stream));
}

// Mask and mirror list of a masked single grid into the workspace; the grid
// descriptor points at them (or at nothing).
hweno_status upload_solid(hweno_ctx* c) {
    hw::Grid2& g = c->hg[0];
    g.solid = nullptr;
    g.sdst = g.ssrc = g.sdir = nullptr;
    g.nsolid = 0;
    g.solid_wall = c->solid_wall;
    for (int k = 0; k < 4; ++k) g.fixed_state[k] = c->fixed_cons[k];
    c->adj.ssrcu = c->adj.sstart = c->adj.sord = nullptr;
    c->adj.nsrc = 0;
    if (c->solid_host.empty()) return HWENO_OK;
    TRY(dev(hipMemcpyAsync(c->solid_dev, c->solid_host.data(), c->solid_host.size(),
                           hipMemcpyHostToDevice, c->stream)));
    const size_t n = c->sdst_host.size();
    if (n) {
        TRY(dev(hipMemcpyAsync(c->sdst_dev, c->sdst_host.data(), n * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
        TRY(dev(hipMemcpyAsync(c->ssrc_dev, c->ssrc_host.data(), n * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
        TRY(dev(hipMemcpyAsync(c->sdir_dev, c->sdir_host.data(), n * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
    }
    g.solid = (const HW_GLOBAL unsigned char*)c->solid_dev;
    g.sdst = (const HW_GLOBAL int*)c->sdst_dev;
    g.ssrc = (const HW_GLOBAL int*)c->ssrc_dev;
    g.sdir = (const HW_GLOBAL int*)c->sdir_dev;
    g.nsolid = (int)n;
    // the reverse mode gathers by mirror source: the entries with a source,
    // grouped by it (ascending source, then list order)
    std::vector<int> ord;
    for (size_t e = 0; e < n; ++e)
        if (c->ssrc_host[e] >= 0) ord.push_back((int)e);
    std::stable_sort(ord.begin(), ord.end(),
                     [&](int a, int b) { return c->ssrc_host[a] < c->ssrc_host[b]; });
    std::vector<int> srcu, start;
    for (size_t k = 0; k < ord.size(); ++k) {
        if (k == 0 || c->ssrc_host[ord[k]] != c->ssrc_host[ord[k - 1]]) {
            srcu.push_back(c->ssrc_host[ord[k]]);
            start.push_back((int)k);
        }
    }
    start.push_back((int)ord.size());
    if (!srcu.empty() && c->ssrcu_dev) {
        TRY(dev(hipMemcpyAsync(c->ssrcu_dev, srcu.data(), srcu.size() * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
        TRY(dev(hipMemcpyAsync(c->sstart_dev, start.data(), start.size() * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
        TRY(dev(hipMemcpyAsync(c->sord_dev, ord.data(), ord.size() * sizeof(int),
                               hipMemcpyHostToDevice, c->stream)));
        c->adj.ssrcu = c->ssrcu_dev;
        c->adj.sstart = c->sstart_dev;
        c->adj.sord = c->sord_dev;
        c->adj.nsrc = (int)srcu.size();
    }
    return dev(hipStreamSynchronize(c->stream));
}

hweno_status upload_state(hweno_ctx* c) {
    TRY(dev(hipMemcpyAsync(c->dst, c->hst.data(), c->hst.size() * sizeof(hw::InstState),
                           hipMemcpyHostToDevice, c->stream)));
    return dev(hipStreamSynchronize(c->stream));
}

hweno_status download_state(hweno_ctx* c) {
    TRY(dev(hipMemcpyAsync(c->hst.data(), c->dst, c->hst.size() * sizeof(hw::InstState),
                           hipMemcpyDeviceToHost, c->stream)));
    return dev(hipStreamSynchronize(c->stream));
}

hw::Grid2& g2(hweno_ctx* c) { return c->hg[0]; }

hweno_status ghost(hweno_ctx* c, int si, int stage = -1) {
    if (c->dim() == 2) {
        if (!c->batch && !c->sdst_host.empty())     // walls inside the grid first
            TRY(dev(hw::launch_solid2(c->dg, (int)c->sdst_host.size(), si, c->stream)));
        return dev(hw::launch_ghost2(c->bl, si, c->stream, c->tm(), stage));
    }
    return dev(hw::launch_ghost1(c->g1, c->S1[si], c->stream, c->tm()));
}

// b: the 2D launch list to use (the stage sets of keep_stages); default the grid's
hweno_status residual(hweno_ctx* c, int si, const hw::BatchL* b = nullptr) {
    if (c->dim() == 2) return dev(hw::launch_residual2(b ? *b : c->bl, si, c->stream, c->tm()));
    return dev(hw::launch_residual1(c->g1, c->S1[si], c->stream, c->tm()));
}

hweno_status update(hweno_ctx* c, int stage, int i0, int iin, int iout, double* R, double* V,
                    const double* src = nullptr, const hw::BatchL* b = nullptr) {
    if (c->dim() == 2)
        return dev(hw::launch_update2(b ? *b : c->bl, stage, i0, iin, iout, R, V, c->stream,
                                      c->tm(), src));
    return dev(hw::launch_update1(c->g1, stage, c->S1[i0], c->S1[iin], c->S1[iout], R, V,
                                  c->stream, c->tm(), src));
}

hweno_status reset(hweno_ctx* c) {
    if (c->dim() == 2) return dev(hw::launch_reset2(c->bl, c->stream));
    return dev(hw::launch_reset(c->red, c->stream));
}

hweno_status read_reduce(hweno_ctx* c, hw::Reduce* r) {
    TRY(dev(hipMemcpyAsync(r, c->red, sizeof(hw::Reduce), hipMemcpyDeviceToHost, c->stream)));
    TRY(dev(hipStreamSynchronize(c->stream)));
    if (c->timer.on) c->timer.collect();
    return HWENO_OK;
}

void fill_diag(double t, const hw::Reduce& r, hweno_diag* d, int restarts, bool stage1_alpha) {
    if (!d) return;
    d->t = t;
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

hweno_status validate(const hweno_grid* grid, const hweno_physics* phys, const hweno_bcs* bcs,
                      const hweno_options* opt) {
    if (!grid || !phys || !bcs || !opt) return HWENO_E_INVAL;
    if (grid->dim != 1 && grid->dim != 2) return HWENO_E_INVAL;
    if (grid->nx < 4 || !(grid->x1 > grid->x0)) return HWENO_E_INVAL;
    if (grid->dim == 2 && (grid->ny < 4 || !(grid->y1 > grid->y0))) return HWENO_E_INVAL;
    if (!(phys->gamma > 1.0) || !(phys->Pr > 0.0) || !(phys->mu_ref >= 0.0) ||
        !(phys->T_ref > 0.0) || !std::isfinite(phys->mu_exp))
        return HWENO_E_INVAL;
    if (!(opt->cfl > 0.0) || !(opt->eps_pp > 0.0) || !(opt->eps_weno > 0.0) ||
        opt->max_halvings < 0 || (opt->keep_stages != 0 && opt->keep_stages != 1) ||
        (opt->gradients != 0 && opt->gradients != 1) ||
        std::isnan(opt->b_visc) || std::isnan(opt->t_final))
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
    return HWENO_OK;
}

// Builds the context of n validated instances (host side only).
hweno_ctx* make_ctx(int n, const hweno_grid* grids, const hweno_physics* phys,
                    const hweno_bcs* bcs, const hweno_options* opts, bool batch) {
    std::unique_ptr<hweno_ctx> owner(new (std::nothrow) hweno_ctx);
    hweno_ctx* c = owner.get();
    if (!c) return nullptr;
    c->batch = batch;
    c->in.resize(n);
    for (int p = 0; p < n; ++p) c->in[p] = Inst{grids[p], phys[p], bcs[p], opts[p]};
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    if (c->dim() == 2) {
        c->hg.assign(n, hw::Grid2{});
        c->hst.assign(n, hw::InstState{});
        c->have.assign(n, 0);
        for (int p = 0; p < n; ++p) {
            hw::Grid2& g = c->hg[p];
            g.nx = grids[p].nx;
            g.ny = grids[p].ny;
            g.NX = g.nx + 2 * HALO;
            g.NY = g.ny + 2 * HALO;
            g.ncell = (long long)g.NX * g.NY;
            g.K = make_consts(c->in[p]);
            for (int s = 0; s < 4; ++s) make_side(c->in[p], s, g.side[s]);
            hw::InstState& st = c->hst[p];
            rule(c->in[p], &st.cfl_h, &st.visc_dt);
            st.t_final = opts[p].t_final;
            st.max_halvings = opts[p].max_halvings;
            st.active = batch ? 0 : 1;       // a single grid is always active
        }
    } else {
        c->g1.K = make_consts(c->in[0]);
        for (int s = 0; s < 2; ++s) make_side(c->in[0], s, c->g1.side[s]);
    }
    c->ws_bytes = layout(c, nullptr);
    return owner.release();
}

// One step of every active instance of a batch (eq. (2.12) with the step rule
// on the device); recorded into a graph by hweno_batch_run.
hweno_status batch_step(const hw::BatchL& b, hipStream_t st) {
    TRY(dev(hw::launch_reset2(b, st)));
    TRY(dev(hw::launch_ghost2(b, 0, st, nullptr)));
    TRY(dev(hw::launch_residual2(b, 0, st, nullptr)));
    TRY(dev(hw::launch_dt2(b, st)));
    TRY(dev(hw::launch_update2(b, 1, 0, 0, 1, nullptr, nullptr, st, nullptr)));
    TRY(dev(hw::launch_ghost2(b, 1, st, nullptr)));
    TRY(dev(hw::launch_residual2(b, 1, st, nullptr)));
    TRY(dev(hw::launch_update2(b, 2, 0, 1, 2, nullptr, nullptr, st, nullptr)));
    TRY(dev(hw::launch_ghost2(b, 2, st, nullptr)));
    TRY(dev(hw::launch_residual2(b, 2, st, nullptr)));
    TRY(dev(hw::launch_update2(b, 3, 0, 2, 1, nullptr, nullptr, st, nullptr)));
    return dev(hw::launch_commit2(b, st));
}

// Records nsteps batch steps on the context's private stream (the caller's
// stream may be the legacy default stream, which cannot be captured); the
// graph is then launched on the caller's stream.
hweno_status capture(hweno_ctx* c, int nsteps, hipGraphExec_t* out) {
    if (!c->cap_stream) TRY(dev(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking)));
    hipGraph_t graph = nullptr;
    hipStream_t user = c->stream;
    TRY(dev(hipStreamSynchronize(user)));
    c->stream = c->cap_stream;
    hweno_status s = dev(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    if (s != HWENO_OK) {
        c->stream = user;
        return s;
    }
    if (c->ngroups == 2) {
        // the second group's chain on a second stream, forked from and
        // joined back into the capturing stream
        hipEvent_t fork = nullptr, join = nullptr;
        if (!c->cap_stream2)
            s = dev(hipStreamCreateWithFlags(&c->cap_stream2, hipStreamNonBlocking));
        if (s == HWENO_OK) s = dev(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
        if (s == HWENO_OK) s = dev(hipEventCreateWithFlags(&join, hipEventDisableTiming));
        if (s == HWENO_OK) s = dev(hipEventRecord(fork, c->stream));
        if (s == HWENO_OK) s = dev(hipStreamWaitEvent(c->cap_stream2, fork, 0));
        for (int k = 0; k < nsteps && s == HWENO_OK; ++k) {
            s = batch_step(c->blg[0], c->stream);
            if (s == HWENO_OK) s = batch_step(c->blg[1], c->cap_stream2);
        }
        if (s == HWENO_OK) s = dev(hipEventRecord(join, c->cap_stream2));
        if (s == HWENO_OK) s = dev(hipStreamWaitEvent(c->stream, join, 0));
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
    } else {
        for (int k = 0; k < nsteps && s == HWENO_OK; ++k) s = batch_step(c->bl, c->stream);
    }
    const hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->stream = user;
    if (s != HWENO_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s;
    }
    TRY(dev(e));
    const hipError_t ei = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    return dev(ei);
}

}  // namespace

extern "C" {

HWENO_API hweno_status hweno_default_options(hweno_options* o) {
    GUARD_BEGIN
    if (!o) return HWENO_E_INVAL;
    o->cfl = 0.6;
    o->b_visc = 0.001;
    o->eps_pp = 1e-12;
    o->eps_weno = 1e-8;
    o->t_final = 0.0;
    o->linear_weights = 0;
    o->max_halvings = 64;
    o->linear_gradients = 0;
    o->keep_stages = 0;
    o->gradients = 0;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_create(const hweno_grid* grid, const hweno_physics* phys,
                                    const hweno_bcs* bcs, const hweno_options* opt,
                                    hweno_ctx** out) {
    GUARD_BEGIN
    if (!out) return HWENO_E_INVAL;
    *out = nullptr;
    TRY(validate(grid, phys, bcs, opt));
    hweno_ctx* c = make_ctx(1, grid, phys, bcs, opt, false);
    if (!c) return HWENO_E_NOMEM;
    *out = c;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_batch_create(int n, const hweno_grid* grids,
                                          const hweno_physics* phys, const hweno_bcs* bcs,
                                          const hweno_options* opts, hweno_ctx** out) {
    GUARD_BEGIN
    if (!out) return HWENO_E_INVAL;
    *out = nullptr;
    if (n < 1 || n > HWENO_BATCH_MAX || !grids || !phys || !bcs || !opts) return HWENO_E_INVAL;
    for (int p = 0; p < n; ++p) {
        TRY(validate(grids + p, phys + p, bcs + p, opts + p));
        if (grids[p].dim != 2) return HWENO_E_INVAL;
        // one launch serves every instance: one gradient scheme per batch
        if (opts[p].gradients != opts[0].gradients) return HWENO_E_INVAL;
    }
    hweno_ctx* c = make_ctx(n, grids, phys, bcs, opts, true);
    if (!c) return HWENO_E_NOMEM;
    *out = c;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_destroy(hweno_ctx* c) {
    GUARD_BEGIN
    if (!c) return HWENO_E_INVAL;
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->cap_stream2) (void)hipStreamDestroy(c->cap_stream2);
    c->timer.destroy();
    delete c;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_workspace_bytes(const hweno_ctx* c, size_t* bytes) {
    GUARD_BEGIN
    if (!c || !bytes) return HWENO_E_INVAL;
    *bytes = c->ws_bytes;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_workspace(hweno_ctx* c, void* p, size_t bytes) {
    GUARD_BEGIN
    if (!c || !p) return HWENO_E_INVAL;
    if (bytes < c->ws_bytes || (reinterpret_cast<uintptr_t>(p) % ALIGN) != 0)
        return HWENO_E_WORKSPACE;
    c->ws = static_cast<char*>(p);
    layout(c, c->ws);
    c->has_state = false;
    c->state_checked = false;
    c->cur = 0;
    std::fill(c->have.begin(), c->have.end(), 0);
    if (c->dim() == 2) {
        for (auto& st : c->hst) {
            st.t = 0.0;
            st.status = 0;
        }
        TRY(upload_state(c));
        if (!c->batch) {
            TRY(upload_profiles(c));
            TRY(upload_solid(c));
        }
        TRY(upload_grids(c));
    }
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_inflow_profile(hweno_ctx* c, int side, const double* prim,
                                                int n) {
    GUARD_BEGIN
    if (!c || c->batch || c->dim() != 2 || side < 0 || side > 3) return HWENO_E_INVAL;
    const Inst& in = c->i0();
    if (in.bcs.kind[side] != HWENO_BC_INFLOW) return HWENO_E_INVAL;
    std::vector<double> cons;
    if (prim) {
        if (n != (side < 2 ? in.grid.ny : in.grid.nx)) return HWENO_E_INVAL;
        const double g = in.phys.gamma;
        cons.resize(4 * (size_t)n);
        for (int k = 0; k < n; ++k) {
            const double r = prim[4 * k], u = prim[4 * k + 1], v = prim[4 * k + 2];
            const double p = prim[4 * k + 3];
            if (!std::isfinite(r) || !std::isfinite(u) || !std::isfinite(v) ||
                !std::isfinite(p) || !(r > 0.0) || !(p > 0.0))
                return HWENO_E_INVAL;
            cons[4 * k] = r;
            cons[4 * k + 1] = r * u;
            cons[4 * k + 2] = r * v;
            cons[4 * k + 3] = p / (g - 1.0) + 0.5 * r * (u * u + v * v);
        }
    }
    c->prof_host[side] = std::move(cons);
    if (!c->ws) return HWENO_OK;
    TRY(upload_profiles(c));
    return upload_grids(c);
    GUARD_END
}

namespace {
// Mirror list of a mask (row-major ny x nx, nonzero = solid): every solid cell
// with a fluid cell within HALO cells in both directions is the mirror image,
// across the nearest wall face along +x, -x, +y, -y (ties in that order), of a
// fluid cell; a mirror off the grid or in solid falls back to the first fluid
// cell in that direction; a cell with fluid only diagonally is left as it is.
// A cell marked in `fixed` (may be null) is listed with source -1: it holds
// the prescribed state instead.
void mirror_list(const unsigned char* m, const unsigned char* fixed, int nx, int ny, int NX,
                 std::vector<int>& dst, std::vector<int>& src, std::vector<int>& dir) {
    auto solid = [&](int j, int i) { return m[(size_t)j * nx + i] != 0; };
    auto in = [&](int j, int i) { return j >= 0 && j < ny && i >= 0 && i < nx; };
    auto ghosted = [&](int j, int i) { return (j + HALO) * NX + i + HALO; };
    const int DJ[4] = {0, 0, 1, -1}, DI[4] = {1, -1, 0, 0};
    for (int j = 0; j < ny; ++j) {
        for (int i = 0; i < nx; ++i) {
            if (!solid(j, i)) continue;
            bool near = false;
            for (int jj = std::max(j - HALO, 0); jj <= std::min(j + HALO, ny - 1) && !near; ++jj)
                for (int ii = std::max(i - HALO, 0); ii <= std::min(i + HALO, nx - 1); ++ii)
                    if (!solid(jj, ii)) {
                        near = true;
                        break;
                    }
            if (!near) continue;
            if (fixed && fixed[(size_t)j * nx + i]) {
                dst.push_back(ghosted(j, i));
                src.push_back(-1);
                dir.push_back(0);
                continue;
            }
            int bk = 0, bd = -1;
            for (int d = 0; d < 4; ++d) {
                int k = 1;
                while (in(j + k * DJ[d], i + k * DI[d]) && solid(j + k * DJ[d], i + k * DI[d])) ++k;
                if (!in(j + k * DJ[d], i + k * DI[d])) continue;
                if (bd < 0 || k < bk) {
                    bk = k;
                    bd = d;
                }
            }
            if (bd < 0) continue;
            int js = j + (2 * bk - 1) * DJ[bd], is = i + (2 * bk - 1) * DI[bd];
            if (!in(js, is) || solid(js, is)) {
                js = j + bk * DJ[bd];
                is = i + bk * DI[bd];
            }
            dst.push_back(ghosted(j, i));
            src.push_back(ghosted(js, is));
            dir.push_back(bd < 2 ? 0 : 1);
        }
    }
}
}  // namespace

HWENO_API hweno_status hweno_set_solid(hweno_ctx* c, const unsigned char* mask, int wall) {
    GUARD_BEGIN
    if (!c || c->batch || c->dim() != 2) return HWENO_E_INVAL;
    const int nx = c->i0().grid.nx, ny = c->i0().grid.ny;
    std::vector<unsigned char> m;
    std::vector<int> dst, src, dir;
    if (mask) {
        if (wall != HWENO_BC_SLIP && wall != HWENO_BC_NOSLIP) return HWENO_E_INVAL;
        m.assign(mask, mask + (size_t)nx * ny);
        for (auto& v : m) v = v ? 1 : 0;
        bool fluid = false;
        for (auto v : m) fluid = fluid || v == 0;
        if (!fluid) return HWENO_E_INVAL;
        mirror_list(m.data(), nullptr, nx, ny, nx + 2 * HALO, dst, src, dir);
    }
    c->fixed_host.clear();
    c->solid_host = std::move(m);
    c->sdst_host = std::move(dst);
    c->ssrc_host = std::move(src);
    c->sdir_host = std::move(dir);
    c->solid_wall = wall;
    if (!c->ws) return HWENO_OK;
    TRY(upload_solid(c));
    return upload_grids(c);
    GUARD_END
}

HWENO_API hweno_status hweno_set_solid_state(hweno_ctx* c, const unsigned char* fixed,
                                             const double* state) {
    GUARD_BEGIN
    if (!c || c->batch || c->dim() != 2 || c->solid_host.empty()) return HWENO_E_INVAL;
    const int nx = c->i0().grid.nx, ny = c->i0().grid.ny;
    std::vector<unsigned char> f;
    double cons[4] = {0.0, 0.0, 0.0, 0.0};
    if (fixed) {
        if (!state) return HWENO_E_INVAL;
        const double r = state[0], u = state[1], v = state[2], p = state[3];
        if (!(r > 0.0) || !(p > 0.0) || !std::isfinite(r) || !std::isfinite(u) ||
            !std::isfinite(v) || !std::isfinite(p))
            return HWENO_E_INVAL;
        f.assign(fixed, fixed + (size_t)nx * ny);
        for (size_t k = 0; k < f.size(); ++k) {
            f[k] = f[k] ? 1 : 0;
            if (f[k] && !c->solid_host[k]) return HWENO_E_INVAL;
        }
        cons[0] = r;
        cons[1] = r * u;
        cons[2] = r * v;
        cons[3] = p / (c->i0().phys.gamma - 1.0) + 0.5 * r * (u * u + v * v);
    }
    std::vector<int> dst, src, dir;
    mirror_list(c->solid_host.data(), fixed ? f.data() : nullptr, nx, ny, nx + 2 * HALO, dst,
                src, dir);
    c->fixed_host = std::move(f);
    for (int k = 0; k < 4; ++k) c->fixed_cons[k] = cons[k];
    c->sdst_host = std::move(dst);
    c->ssrc_host = std::move(src);
    c->sdir_host = std::move(dir);
    if (!c->ws) return HWENO_OK;
    TRY(upload_solid(c));
    return upload_grids(c);
    GUARD_END
}

HWENO_API hweno_status hweno_set_stream(hweno_ctx* c, void* s) {
    GUARD_BEGIN
    if (!c) return HWENO_E_INVAL;
    c->stream = static_cast<hipStream_t>(s);
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_state(hweno_ctx* c, const double* U, double t) {
    GUARD_BEGIN
    if (!c || !U || !std::isfinite(t) || c->batch) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->dim() == 2) TRY(dev(hw::launch_copy_in2(g2(c), U, g2(c).S[c->cur], c->stream)));
    else TRY(dev(hw::launch_copy_in1(c->g1, U, c->S1[0], c->stream)));
    c->t = t;
    c->has_state = true;
    c->state_checked = false;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_get_state(hweno_ctx* c, double* U, double* t) {
    GUARD_BEGIN
    if (!c || !U || c->batch) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    if (c->dim() == 2) TRY(dev(hw::launch_copy_out2(g2(c), g2(c).S[c->cur], U, c->stream)));
    else TRY(dev(hw::launch_copy_out1(c->g1, c->S1[0], U, c->stream)));
    if (t) *t = c->t;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_residual(hweno_ctx* c, const double* U, double* R, double* V,
                                      hweno_diag* diag) {
    GUARD_BEGIN
    if (!c || !U || !R || !V || c->batch) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->dim() == 2) TRY(dev(hw::launch_copy_in2(g2(c), U, g2(c).S[2], c->stream)));
    else TRY(dev(hw::launch_copy_in1(c->g1, U, c->S1[2], c->stream)));
    TRY(reset(c));
    TRY(ghost(c, 2));
    TRY(residual(c, 2));
    TRY(update(c, 0, 2, 2, 2, R, V));
    if (diag) {
        hw::Reduce r;
        TRY(read_reduce(c, &r));
        fill_diag(c->t, r, diag, 0, false);
        diag->dt = 0.0;
        diag->min_rho = diag->min_p = NAN;
    }
    return HWENO_OK;
    GUARD_END
}

}  // extern "C"

namespace {

static_assert(hw::STATIC_SCRATCH_BYTES == HWENO_NOALLOC_BYTES,
              "the static scratch and its documented size differ");

// Residual-only carve of the static scratch for a 2D grid: descriptor,
// instance state, reduction slots, block table, one ghosted state and the
// intermediates of one residual (no RK buffers, reverse-mode or profile
// arrays).  base == nullptr: size only.
size_t static_layout2(hw::Grid2& g, char* base, hw::Grid2** dgrid, hw::InstState** dst,
                      int** dstart) {
    size_t off = 0;
    auto take_bytes = [&](size_t nb) -> char* {
        char* p = base ? base + off : nullptr;
        off += up(nb);
        return p;
    };
    auto take = [&](size_t nd) -> hw::gdouble* {
        return (hw::gdouble*)take_bytes(nd * sizeof(double));
    };
    const size_t m = (size_t)g.ncell;
    *dgrid = reinterpret_cast<hw::Grid2*>(take_bytes(sizeof(hw::Grid2)));
    *dst = reinterpret_cast<hw::InstState*>(take_bytes(sizeof(hw::InstState)));
    g.st = (HW_GLOBAL hw::InstState*)*dst;
    g.red = (HW_GLOBAL hw::Reduce*)take_bytes(sizeof(hw::Reduce));
    *dstart = reinterpret_cast<int*>(take_bytes(2 * hw::KB_COUNT * sizeof(int)));
    hw::gdouble* S = take(12 * m);
    for (int k = 0; k < 4; ++k) g.S[k] = S;
    g.xf = take(24 * m);
    g.yf = take(24 * m);
    g.xv = g.yv = nullptr;   // the full volume values are the reverse mode's
    g.vc = take(2 * hw::VC_B * m);
    g.wb = take(6 * m);
    g.vk = take(8 * m);
    g.vn = take(8 * m);
    g.rb = take(18 * m);
    g.gf = take(36 * m);
    g.vf = take(8 * m);
    g.fx = take(8 * m);
    g.fy = take(8 * m);
    g.solid = nullptr;
    g.sdst = g.ssrc = g.sdir = nullptr;
    g.nsolid = 0;
    for (int sd = 0; sd < 4; ++sd) g.side[sd].prof = g.side[sd].prof_stage = nullptr;
    return off;
}

// The same for a 1D grid: reduction slots, one ghosted state, intermediates.
size_t static_layout1(hw::Grid1& g, char* base, double** S) {
    size_t off = 0;
    auto take_bytes = [&](size_t nb) -> char* {
        char* p = base ? base + off : nullptr;
        off += up(nb);
        return p;
    };
    auto take = [&](size_t nd) -> hw::gdouble* {
        return (hw::gdouble*)take_bytes(nd * sizeof(double));
    };
    const size_t m = (size_t)g.NX;
    g.red = (HW_GLOBAL hw::Reduce*)take_bytes(sizeof(hw::Reduce));
    *S = (double*)take(6 * m);
    g.pts = take(12 * m);
    g.wb = take(2 * m);
    g.vk = take(3 * m);
    g.vn = take(3 * m);
    g.rb = take(4 * m);
    g.gr = take(8 * m);
    g.fh = take(3 * m);
    g.vf = take(3 * m);
    return off;
}

}  // namespace

extern "C" {

HWENO_API hweno_status hweno_residual_noalloc(hweno_ctx* c, const double* U, double* R,
                                              double* V, hweno_diag* diag) {
    GUARD_BEGIN
    if (!c || !U || !R || !V || c->batch) return HWENO_E_INVAL;
    // inflow profiles and masks live in the context's workspace
    if (!c->solid_host.empty()) return HWENO_E_INVAL;
    for (int sd = 0; sd < 4; ++sd)
        if (!c->prof_host[sd].empty() || !c->stage_host[sd].empty()) return HWENO_E_INVAL;
    hipStream_t st = c->stream;
    hw::Reduce* red = nullptr;
    if (c->dim() == 2) {
        hw::Grid2 g = c->hg[0];
        hw::Grid2* dg = nullptr;
        hw::InstState* dst = nullptr;
        int* dstart = nullptr;
        if (static_layout2(g, nullptr, &dg, &dst, &dstart) > hw::STATIC_SCRATCH_BYTES)
            return HWENO_E_WORKSPACE;
        void* base = nullptr;
        TRY(dev(hw::static_scratch(&base)));
        static_layout2(g, static_cast<char*>(base), &dg, &dst, &dstart);
        c->sgrid = g;
        c->sstate = hw::InstState{};
        c->sstate.active = 1;
        hw::batch_blocks(&c->sgrid, 1, c->tiles, c->sstart);
        TRY(dev(hipMemcpyAsync(dg, &c->sgrid, sizeof(hw::Grid2), hipMemcpyHostToDevice, st)));
        TRY(dev(hipMemcpyAsync(dst, &c->sstate, sizeof(hw::InstState), hipMemcpyHostToDevice,
                               st)));
        TRY(dev(hipMemcpyAsync(dstart, c->sstart, sizeof(c->sstart), hipMemcpyHostToDevice,
                               st)));
        hw::BatchL bl;
        bl.dg = dg;
        bl.dstart = dstart;
        bl.hstart = c->sstart;
        bl.n = 1;
        bl.tiles = c->tiles;
        bl.var_mu = c->i0().phys.mu_exp != 0.0;
        bl.dr = c->i0().opt.gradients != 0;
        TRY(dev(hw::launch_copy_in2(g, U, g.S[0], st)));
        TRY(dev(hw::launch_reset2(bl, st)));
        TRY(dev(hw::launch_ghost2(bl, 0, st, nullptr)));
        TRY(dev(hw::launch_residual2(bl, 0, st, nullptr)));
        TRY(dev(hw::launch_update2(bl, 0, 0, 0, 0, R, V, st, nullptr)));
        red = (hw::Reduce*)g.red;
    } else {
        hw::Grid1 g = c->g1;
        double* S = nullptr;
        if (static_layout1(g, nullptr, &S) > hw::STATIC_SCRATCH_BYTES) return HWENO_E_WORKSPACE;
        void* base = nullptr;
        TRY(dev(hw::static_scratch(&base)));
        static_layout1(g, static_cast<char*>(base), &S);
        red = (hw::Reduce*)g.red;
        TRY(dev(hw::launch_copy_in1(g, U, S, st)));
        TRY(dev(hw::launch_reset(red, st)));
        TRY(dev(hw::launch_ghost1(g, S, st, nullptr)));
        TRY(dev(hw::launch_residual1(g, S, st, nullptr)));
        TRY(dev(hw::launch_update1(g, 0, S, S, S, R, V, st, nullptr)));
    }
    if (diag) {
        hw::Reduce r;
        TRY(dev(hipMemcpyAsync(&r, red, sizeof(hw::Reduce), hipMemcpyDeviceToHost, st)));
        TRY(dev(hipStreamSynchronize(st)));
        fill_diag(c->t, r, diag, 0, false);
        diag->dt = 0.0;
        diag->min_rho = diag->min_p = NAN;
    }
    return HWENO_OK;
    GUARD_END
}

}  // extern "C"

namespace {

// One SSP-RK3 step of a single grid (eq. (2.12)); src[k] (may be null) are
// source moments added to the residual of stage k+1; `staged`: the ghost fill
// of stage k+1 takes the sides' stage-k+1 inflow profiles.  With sources or
// staged inflow the step size is fixed and a rejected stage is an error
// instead of a restart.
hweno_status step(hweno_ctx* c, double dt, const double* const* src, hweno_diag* diag,
                  bool staged = false) {
    const bool two = c->dim() == 2;
    const bool auto_dt = !(dt > 0.0);
    double cfl_h, visc;
    rule(c->i0(), &cfl_h, &visc);
    const double t_left = c->i0().opt.t_final > 0.0 ? c->i0().opt.t_final - c->t : INFINITY;
    if (auto_dt && !(t_left > 0.0)) {   // already at t_final: nothing to do
        if (diag) {
            std::memset(diag, 0, sizeof(*diag));
            diag->t = c->t;
        }
        return HWENO_OK;
    }
    const int max_halvings = (src || staged) ? 0 : c->i0().opt.max_halvings;
    // state buffers: 2D by index into Grid2::S (the current one is `cur`);
    // 1D by index into S1 with S1[0] current
    const int a = two ? c->cur : 0, b = two ? 1 - c->cur : 1, s2 = 2;
    const double* src1 = src ? src[0] : nullptr;
    const double* src2 = src ? src[1] : nullptr;
    const double* src3 = src ? src[2] : nullptr;
    double cur_dt = dt;
    int restarts = 0;
    hw::Reduce r;
    for (;;) {
        TRY(reset(c));
        // the input state is checked once: the output of an accepted step
        // already passed the same test in the stage-3 update
        if (restarts == 0 && !c->state_checked) {
            if (two) TRY(dev(hw::launch_check2(c->bl, a, c->stream)));
            else TRY(dev(hw::launch_check1(c->g1, c->S1[0], c->stream)));
        }
        TRY(ghost(c, a, staged ? 0 : -1));
        TRY(residual(c, a));
        if (auto_dt && restarts == 0)
            TRY(dev(hw::launch_dt(c->red, cfl_h, visc, t_left, c->stream)));
        else
            TRY(dev(hw::launch_set_dt(c->red, cur_dt, c->stream)));
        TRY(update(c, 1, a, a, b, nullptr, nullptr, src1));
        TRY(ghost(c, b, staged ? 1 : -1));
        TRY(residual(c, b));
        TRY(update(c, 2, a, b, s2, nullptr, nullptr, src2));
        TRY(ghost(c, s2, staged ? 2 : -1));
        TRY(residual(c, s2));
        TRY(update(c, 3, a, s2, b, nullptr, nullptr, src3));
        TRY(read_reduce(c, &r));
        if (restarts == 0 && r.bad[0] != 0) return HWENO_E_NONFINITE;
        if (!(r.dt > 0.0) || !std::isfinite(r.dt)) return HWENO_E_NONFINITE;
        if (r.bad[1] == 0 && r.bad[2] == 0 && r.bad[3] == 0) break;
        if (restarts >= max_halvings) return HWENO_E_INADMISSIBLE;
        ++restarts;
        cur_dt = 0.5 * r.dt;
    }
    if (two) c->cur = b;
    else std::swap(c->S1[0], c->S1[1]);
    c->state_checked = true;
    c->t += r.dt;
    fill_diag(c->t, r, diag, restarts, true);
    return HWENO_OK;
}

}  // namespace

extern "C" {

HWENO_API hweno_status hweno_rk_step(hweno_ctx* c, double dt, hweno_diag* diag) {
    GUARD_BEGIN
    if (!c || std::isnan(dt) || c->batch) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    return step(c, dt, nullptr, diag);
    GUARD_END
}

HWENO_API hweno_status hweno_rk_step_source(hweno_ctx* c, double dt, const double* src1,
                                            const double* src2, const double* src3,
                                            hweno_diag* diag) {
    GUARD_BEGIN
    if (!c || !(dt > 0.0) || !std::isfinite(dt) || c->batch || !src1 || !src2 || !src3)
        return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    const double* src[3] = {src1, src2, src3};
    return step(c, dt, src, diag);
    GUARD_END
}

HWENO_API hweno_status hweno_set_inflow_stages(hweno_ctx* c, int side, const double* prim1,
                                               const double* prim2, const double* prim3, int n) {
    GUARD_BEGIN
    if (!c || c->batch || c->dim() != 2 || side < 0 || side > 3) return HWENO_E_INVAL;
    const Inst& in = c->i0();
    if (in.bcs.kind[side] != HWENO_BC_INFLOW) return HWENO_E_INVAL;
    std::vector<double> cons;
    if (prim1 || prim2 || prim3) {
        if (!prim1 || !prim2 || !prim3 || n != (side < 2 ? in.grid.ny : in.grid.nx))
            return HWENO_E_INVAL;
        const double g = in.phys.gamma;
        cons.resize(12 * (size_t)n);
        const double* P[3] = {prim1, prim2, prim3};
        for (int st = 0; st < 3; ++st) {
            for (int k = 0; k < n; ++k) {
                const double* q = P[st] + 4 * k;
                const double r = q[0], u = q[1], v = q[2], p = q[3];
                if (!std::isfinite(r) || !std::isfinite(u) || !std::isfinite(v) ||
                    !std::isfinite(p) || !(r > 0.0) || !(p > 0.0))
                    return HWENO_E_INVAL;
                double* o = cons.data() + 4 * ((size_t)st * n + k);
                o[0] = r;
                o[1] = r * u;
                o[2] = r * v;
                o[3] = p / (g - 1.0) + 0.5 * r * (u * u + v * v);
            }
        }
    }
    c->stage_host[side] = std::move(cons);
    if (!c->ws) return HWENO_OK;
    TRY(upload_profiles(c));
    return upload_grids(c);
    GUARD_END
}

HWENO_API hweno_status hweno_rk_step_inflow(hweno_ctx* c, double dt, hweno_diag* diag) {
    GUARD_BEGIN
    if (!c || !(dt > 0.0) || !std::isfinite(dt) || c->batch || c->dim() != 2)
        return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->has_state) return HWENO_E_STATE;
    return step(c, dt, nullptr, diag, true);
    GUARD_END
}

HWENO_API hweno_status hweno_residual_vjp(hweno_ctx* c, const double* U, const double* Rbar,
                                          const double* Vbar, double* Ubar, double* mu_bar) {
    GUARD_BEGIN
    if (!c || !U || !Rbar || !Ubar || c->batch) return HWENO_E_INVAL;
    if (c->i0().opt.gradients != 0) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->dim() == 1) {   // the step's stage buffer 2 holds U (the state is kept)
        TRY(dev(hw::launch_copy_in1(c->g1, U, c->S1[2], c->stream)));
        TRY(reset(c));
        TRY(ghost(c, 2));
        TRY(residual(c, 2));
        hw::AdjIn A{Rbar, Vbar, 1.0, 1.0};
        TRY(dev(hw::launch_vjp1(c->g1, A, c->adj1, c->S1[2], Ubar, c->mu_dev, 0, c->stream)));
        if (mu_bar) {
            TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream)));
            TRY(dev(hipStreamSynchronize(c->stream)));
        }
        return HWENO_OK;
    }
    const hw::Grid2& g = g2(c);
    hw::BatchL full = c->bl;   // the adjoint kernels read all six face gradients
    full.full_grad = true;
    TRY(dev(hw::launch_copy_in2(g, U, g.S[2], c->stream)));
    TRY(reset(c));
    TRY(ghost(c, 2));
    TRY(residual(c, 2, &full));
    hw::AdjIn A{Rbar, Vbar, 1.0, 1.0};
    TRY(dev(hw::launch_vjp2(g, A, c->adj, g.S[2], Ubar, c->mu_dev, 0, c->stream)));
    if (mu_bar) {
        TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                               c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
    }
    return HWENO_OK;
    GUARD_END
}

// Reverse mode of one SSP-RK3 step with the step size frozen (eq. (2.12)):
//   U1 = B(U0) + dt F(U0),  U2 = 3/4 B(U0) + 1/4 (B(U1) + dt F(U1)),
//   U3 = 1/3 B(U0) + 2/3 (B(U2) + dt F(U2)),   B(U) = (ubar, hat-v(U)).
// The stages are recomputed from U0 with the forward kernels, then the three
// residual adjoints run in reverse with the stage cotangents as seeds.
HWENO_API hweno_status hweno_rk_step_vjp(hweno_ctx* c, const double* U0, double dt,
                                         const double* U3bar, double* U0bar, double* mu_bar) {
    GUARD_BEGIN
    if (!c || !U0 || !U3bar || !U0bar || !(dt > 0.0) || !std::isfinite(dt) || c->batch)
        return HWENO_E_INVAL;
    if (c->i0().opt.gradients != 0) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->dim() == 1) {
        // U0, U1, U2 in stage buffers 2, 3, 4 (the state in buffer 0 is kept);
        // every stage adjoint recomputes its residual's intermediates first
        const long long na = 3LL * c->g1.nx, nall = 6LL * c->g1.nx;
        const int ia = 2, ib = 3, ic = 4;
        TRY(dev(hw::launch_copy_in1(c->g1, U0, c->S1[ia], c->stream)));
        TRY(reset(c));
        TRY(dev(hw::launch_set_dt(c->red, dt, c->stream)));
        TRY(ghost(c, ia));
        TRY(residual(c, ia));
        TRY(update(c, 1, ia, ia, ib, nullptr, nullptr));
        TRY(ghost(c, ib));
        TRY(residual(c, ib));
        TRY(update(c, 2, ia, ib, ic, nullptr, nullptr));
        auto vjp_at1 = [&](int si, const double* Rb, const double* Vb, double rs, double vs,
                           double* out, int acc) {
            TRY(reset(c));
            TRY(ghost(c, si));
            TRY(residual(c, si));
            hw::AdjIn A{Rb, Vb, rs, vs};
            return dev(hw::launch_vjp1(c->g1, A, c->adj1, c->S1[si], out, c->mu_dev, acc,
                                       c->stream));
        };
        TRY(vjp_at1(ic, U3bar, U3bar + na, (2.0 / 3.0) * dt, 2.0 / 3.0, c->X2, 0));
        TRY(dev(hw::launch_axpy(c->X2, U3bar, 2.0 / 3.0, na, c->stream)));           // U2bar
        TRY(vjp_at1(ib, c->X2, c->X2 + na, 0.25 * dt, 0.25, c->X1, 1));
        TRY(dev(hw::launch_axpy(c->X1, c->X2, 0.25, na, c->stream)));                // U1bar
        TRY(dev(hw::launch_lin3(c->X2, U3bar, 1.0 / 3.0, 0.75, c->X1, nall, c->stream)));
        TRY(vjp_at1(ia, c->X1, c->X2 + na, dt, 1.0, U0bar, 1));
        TRY(dev(hw::launch_axpy(U0bar, c->X2, 1.0, na, c->stream)));
        if (mu_bar) {
            TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                                   c->stream)));
            TRY(dev(hipStreamSynchronize(c->stream)));
        }
        return HWENO_OK;
    }
    const hw::Grid2& g = g2(c);
    const long long nint = (long long)g.nx * g.ny;
    const int ia = 1 - c->cur, ib = 2, ic = 3;   // U0, U1, U2 (the current state is kept)
    // forward recomputation of the two intermediate stages
    TRY(dev(hw::launch_copy_in2(g, U0, g.S[ia], c->stream)));
    TRY(reset(c));
    TRY(dev(hw::launch_set_dt(c->red, dt, c->stream)));
    // with keep_stages the residual intermediates of U0 stay in the grid's
    // set, those of U1 go to stage set 0 and those of U2 to stage set 1, so
    // the adjoints of stages 2 and 1 need no recomputation
    const bool keep = c->dstage != nullptr;
    // every residual here feeds an adjoint, which reads all six face gradients
    hw::BatchL full = c->bl, full_st[2] = {c->blstage[0], c->blstage[1]};
    full.full_grad = full_st[0].full_grad = full_st[1].full_grad = true;
    const hw::BatchL* b1 = keep ? &full_st[0] : &full;
    TRY(ghost(c, ia));
    TRY(residual(c, ia, &full));
    TRY(update(c, 1, ia, ia, ib, nullptr, nullptr, nullptr, &full));
    TRY(ghost(c, ib));
    TRY(residual(c, ib, b1));
    TRY(update(c, 2, ia, ib, ic, nullptr, nullptr, nullptr, b1));
    // adjoint at stage input si with the intermediates described by gi
    // (launched through bi when they are formed first)
    auto vjp_at = [&](int si, const hw::Grid2& gi, const hw::BatchL* bi, bool form,
                      const double* Rb, const double* Vb, double rs, double vs, double* out,
                      int acc, const double* add, double add_a, const double* pass) {
        if (form) {
            TRY(reset(c));
            TRY(ghost(c, si));
            TRY(residual(c, si, bi));
        }
        hw::AdjIn A{Rb, Vb, rs, vs};
        return dev(hw::launch_vjp2(gi, A, c->adj, g.S[si], out, c->mu_dev, acc, c->stream, add,
                                   add_a, pass));
    };
    // stage 3: seeds 2/3 dt U3bar (residual) and 2/3 U3bar (modified
    // moments); the averages' direct path 2/3 U3bar joins the output (U2bar)
    // (a masked grid's solid cells pass each stage's output adjoint through)
    TRY(vjp_at(ic, keep ? c->stage[1] : g, keep ? &full_st[1] : &full, true, U3bar,
               U3bar + 4 * nint, (2.0 / 3.0) * dt, 2.0 / 3.0, c->X2, 0, U3bar, 2.0 / 3.0,
               U3bar));
    // stage 2: seeds 1/4 dt U2bar and 1/4 U2bar, plus 1/4 U2bar direct (U1bar)
    TRY(vjp_at(ib, keep ? c->stage[0] : g, &full, !keep, c->X2, c->X2 + 4 * nint, 0.25 * dt,
               0.25, c->X1, 1, c->X2, 0.25, c->X2));
    // B(U0)-bar = 1/3 U3bar + 3/4 U2bar + U1bar (into X2)
    TRY(dev(hw::launch_lin3(c->X2, U3bar, 1.0 / 3.0, 0.75, c->X1, 12 * nint, c->stream)));
    // stage 1: residual seed dt U1bar, modified-moment seed B(U0)-bar, plus
    // B(U0)-bar's averages direct
    TRY(vjp_at(ia, g, &full, !keep, c->X1, c->X2 + 4 * nint, dt, 1.0, U0bar, 1, c->X2, 1.0,
               c->X1));
    if (mu_bar) {
        TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                               c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
    }
    return HWENO_OK;
    GUARD_END
}

// ---------------------------------------------------------------------------
// Recorded steps: the step adjoint from a recording instead of a recomputation
// ---------------------------------------------------------------------------
HWENO_API hweno_status hweno_record_bytes(const hweno_ctx* c, int nslots, size_t* bytes) {
    GUARD_BEGIN
    if (!c || !bytes || c->batch || c->dim() != 2 || nslots < 0) return HWENO_E_INVAL;
    *bytes = record_layout(c, nullptr, nslots, nullptr, nullptr);
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_record(hweno_ctx* c, void* buffer, size_t bytes, int nslots) {
    GUARD_BEGIN
    if (!c || c->batch || c->dim() != 2 || nslots < 0) return HWENO_E_INVAL;
    if (nslots > 0 && !buffer) return HWENO_E_INVAL;
    if (nslots > 0 && bytes < record_layout(c, nullptr, nslots, nullptr, nullptr))
        return HWENO_E_WORKSPACE;
    c->rec_base = nslots > 0 ? static_cast<char*>(buffer) : nullptr;
    c->rec_slots = nslots;
    c->rec_desc.clear();
    c->rec_ddesc = nullptr;
    c->rec_dt.assign((size_t)nslots, 0.0);
    if (!c->ws || nslots == 0) return HWENO_OK;
    return upload_record(c);
    GUARD_END
}

HWENO_API hweno_status hweno_rk_step_record(hweno_ctx* c, int slot, const double* U0, double dt,
                                            double* U3) {
    GUARD_BEGIN
    if (!c || !U0 || !U3 || c->batch || c->dim() != 2 || !(dt > 0.0) || !std::isfinite(dt))
        return HWENO_E_INVAL;
    if (c->i0().opt.gradients != 0) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (slot < 0 || slot >= c->rec_slots || c->rec_desc.empty()) return HWENO_E_INVAL;
    const hw::Grid2* dd = c->rec_ddesc + 3 * (size_t)slot;
    const hw::Grid2& d0 = c->rec_desc[3 * (size_t)slot];
    hw::BatchL b[3];
    for (int k = 0; k < 3; ++k) {
        b[k] = c->bl;
        b[k].dg = dd + k;
        b[k].full_grad = true;   // the step adjoint reads all six face gradients
    }
    c->rec_dt[slot] = 0.0;
    TRY(dev(hw::launch_copy_in2(d0, U0, d0.S[0], c->stream)));
    TRY(reset(c));
    TRY(dev(hw::launch_set_dt(c->red, dt, c->stream)));
    const int nsolid = (int)c->sdst_host.size();
    for (int k = 0; k < 3; ++k) {   // stage k + 1 from input S[k] into S[k + 1]
        // walls inside the grid first (the slot's stage input, in place)
        if (nsolid) TRY(dev(hw::launch_solid2(dd + k, nsolid, k, c->stream)));
        TRY(dev(hw::launch_ghost2(b[k], k, c->stream, c->tm())));
        TRY(residual(c, k, &b[k]));
        TRY(update(c, k + 1, 0, k, k + 1, nullptr, nullptr, nullptr, &b[k]));
    }
    TRY(dev(hw::launch_copy_out2(d0, d0.S[3], U3, c->stream)));
    c->rec_dt[slot] = dt;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_rk_step_vjp_recorded(hweno_ctx* c, int slot, const double* U3bar,
                                                  double* U0bar, double* mu_bar) {
    GUARD_BEGIN
    if (!c || !U3bar || !U0bar || c->batch || c->dim() != 2) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (slot < 0 || slot >= c->rec_slots || c->rec_desc.empty() || !(c->rec_dt[slot] > 0.0))
        return HWENO_E_INVAL;
    const double dt = c->rec_dt[slot];
    const hw::Grid2* d = &c->rec_desc[3 * (size_t)slot];
    const long long nint = (long long)d[0].nx * d[0].ny;
    // the stage adjoints in reverse, seeded as in hweno_rk_step_vjp
    hw::AdjIn A3{U3bar, U3bar + 4 * nint, (2.0 / 3.0) * dt, 2.0 / 3.0};
    // mu_bar NULL: this step's mu adjoint joins the device-side running sum
    // (a masked grid's solid cells pass each stage's output adjoint through)
    TRY(dev(hw::launch_vjp2(d[2], A3, c->adj, d[2].S[2], c->X2, c->mu_dev, mu_bar ? 0 : 1,
                            c->stream, U3bar, 2.0 / 3.0, U3bar)));                  // U2bar
    hw::AdjIn A2{c->X2, c->X2 + 4 * nint, 0.25 * dt, 0.25};
    TRY(dev(hw::launch_vjp2(d[1], A2, c->adj, d[1].S[1], c->X1, c->mu_dev, 1, c->stream, c->X2,
                            0.25, c->X2)));                                         // U1bar
    TRY(dev(hw::launch_lin3(c->X2, U3bar, 1.0 / 3.0, 0.75, c->X1, 12 * nint, c->stream)));
    hw::AdjIn A1{c->X1, c->X2 + 4 * nint, dt, 1.0};
    TRY(dev(hw::launch_vjp2(d[0], A1, c->adj, d[0].S[0], U0bar, c->mu_dev, 1, c->stream, c->X2,
                            1.0, c->X1)));
    if (mu_bar) {
        TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost,
                               c->stream)));
        TRY(dev(hipStreamSynchronize(c->stream)));
    }
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_take_mu_bar(hweno_ctx* c, double* mu_bar) {
    GUARD_BEGIN
    if (!c || !mu_bar || c->batch) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    static const double zero = 0.0;
    TRY(dev(hipMemcpyAsync(mu_bar, c->mu_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream)));
    TRY(dev(hipMemcpyAsync(c->mu_dev, &zero, sizeof(double), hipMemcpyHostToDevice, c->stream)));
    return dev(hipStreamSynchronize(c->stream));
    GUARD_END
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
HWENO_API hweno_status hweno_batch_set_state(hweno_ctx* c, int i, const double* U, double t) {
    GUARD_BEGIN
    if (!c || !c->batch || !U || i < 0 || i >= (int)c->in.size() || !std::isfinite(t))
        return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    const hw::Grid2& g = c->hg[i];
    TRY(dev(hw::launch_copy_in2(g, U, g.S[0], c->stream)));
    TRY(download_state(c));
    c->hst[i].t = t;
    c->hst[i].status = 0;
    c->hst[i].halvings = 0;
    TRY(upload_state(c));
    c->have[i] = 1;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_batch_get_state(hweno_ctx* c, int i, double* U, double* t) {
    GUARD_BEGIN
    if (!c || !c->batch || !U || i < 0 || i >= (int)c->in.size()) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (!c->have[i]) return HWENO_E_STATE;
    const hw::Grid2& g = c->hg[i];
    TRY(dev(hw::launch_copy_out2(g, g.S[0], U, c->stream)));
    if (t) *t = c->hst[i].t;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_batch_run(hweno_ctx* c, int nsteps) {
    GUARD_BEGIN
    if (!c || !c->batch || nsteps < 1) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    const int n = (int)c->in.size();
    for (int p = 0; p < n; ++p)
        if (!c->have[p]) return HWENO_E_STATE;
    // run set-up: counters, activity, input admissibility
    TRY(download_state(c));
    int max_halv = 0;
    for (auto& st : c->hst) {
        st.steps = 0;
        st.target = nsteps;
        st.halvings = 0;
        st.restarts = 0;
        st.pp_cells = 0;
        st.active = st.status == 0 && (st.t_final <= 0.0 || st.t < st.t_final);
        max_halv = std::max(max_halv, st.max_halvings);
    }
    TRY(upload_state(c));
    TRY(dev(hw::launch_reset2(c->bl, c->stream)));
    TRY(dev(hw::launch_check2(c->bl, 0, c->stream)));
    std::vector<hw::Reduce> rr(n);
    TRY(dev(hipMemcpyAsync(rr.data(), c->red, n * sizeof(hw::Reduce), hipMemcpyDeviceToHost,
                           c->stream)));
    TRY(dev(hipStreamSynchronize(c->stream)));
    bool bad_input = false;
    for (int p = 0; p < n; ++p) {
        if (c->hst[p].active && rr[p].bad[0] != 0) {
            c->hst[p].status = HWENO_E_NONFINITE;
            c->hst[p].active = 0;
            bad_input = true;
        }
    }
    if (bad_input) TRY(upload_state(c));
    // the whole run as one graph launch
    if (!c->gexec || c->gsteps != nsteps) {
        if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        TRY(capture(c, nsteps, &c->gexec));
        c->gsteps = nsteps;
    }
    hw::Timer* tm = c->tm();
    hw::tbeg(tm, hw::KC_OTHER, c->stream);
    TRY(dev(hipGraphLaunch(c->gexec, c->stream)));
    hw::tend(tm, c->stream);
    TRY(download_state(c));
    if (tm) tm->collect();
    // instances that needed restarts: one more attempt per launch until done
    const long long limit = (long long)nsteps * (max_halv + 1);
    for (long long k = 0; k < limit; ++k) {
        bool any = false;
        for (auto& st : c->hst) any = any || st.active;
        if (!any) break;
        if (!c->gexec1) TRY(capture(c, 1, &c->gexec1));
        TRY(dev(hipGraphLaunch(c->gexec1, c->stream)));
        TRY(download_state(c));
    }
    for (auto& st : c->hst)
        if (st.status != 0) return (hweno_status)st.status;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_batch_get_diag(hweno_ctx* c, int i, hweno_diag* d) {
    GUARD_BEGIN
    if (!c || !c->batch || !d || i < 0 || i >= (int)c->in.size()) return HWENO_E_INVAL;
    const hw::InstState& st = c->hst[i];
    d->t = st.t;
    d->dt = st.dt_last;
    d->alpha_star = st.alpha;
    d->beta_max = st.beta_max;
    d->min_rho = st.min_rho;
    d->min_p = st.min_p;
    d->pp_cells = st.pp_cells;
    d->restarts = (int)st.restarts;
    d->pad = st.steps;
    return HWENO_OK;
    GUARD_END
}

// ---------------------------------------------------------------------------
// Tiles and the autotuner (2D contexts)
// ---------------------------------------------------------------------------
HWENO_API hweno_status hweno_get_tiles(const hweno_ctx* c, hweno_tiles* t) {
    GUARD_BEGIN
    if (!c || !t || c->dim() != 2) return HWENO_E_INVAL;
    t->recon = c->tiles.recon;
    t->grad = c->tiles.grad;
    t->flux = c->tiles.flux;
    t->order = c->order_mode;
    t->xcd = c->tiles.xcd;
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_tiles(hweno_ctx* c, const hweno_tiles* t) {
    GUARD_BEGIN
    if (!c || !t || c->dim() != 2) return HWENO_E_INVAL;
    if ((t->recon != 16 && t->recon != 32) || (t->grad != 0 && t->grad != 32 && t->grad != 64) ||
        (t->flux != 0 && t->flux != 64 && t->flux != 128) || (t->order != 0 && t->order != 1) ||
        (t->xcd != 0 && t->xcd != 1))
        return HWENO_E_INVAL;
    c->tiles.recon = t->recon;
    c->tiles.grad = t->grad;
    c->tiles.flux = t->flux;
    c->tiles.xcd = t->xcd;
    c->order_mode = t->order;
    if (!c->ws) return HWENO_OK;
    return upload_grids(c);
    GUARD_END
}

HWENO_API hweno_status hweno_autotune(hweno_ctx* c, int reps, hweno_tiles* chosen) {
    GUARD_BEGIN
    if (!c || c->dim() != 2 || reps < 1) return HWENO_E_INVAL;
    if (!c->ws) return HWENO_E_WORKSPACE;
    if (c->batch) {
        for (char h : c->have)
            if (!h) return HWENO_E_STATE;
    } else if (!c->has_state) {
        return HWENO_E_STATE;
    }
    if (!c->timer.init()) return HWENO_E_DEVICE;
    const bool was_on = c->timer.on;
    const unsigned was_mask = c->timer.mask;
    const int si = c->batch ? 0 : c->cur;
    if (c->batch) {
        // every instance active for the timing passes
        TRY(download_state(c));
        for (auto& st : c->hst) st.active = 1;
        TRY(upload_state(c));
    }
    // `reps` residual evaluations of the current states, each followed by a
    // stage-1 update into the scratch state S[2] (the fluxes may be formed
    // there); ms per kernel class
    auto one = [&]() -> hweno_status {
        TRY(reset(c));
        TRY(ghost(c, si));
        TRY(residual(c, si));
        TRY(dev(hw::launch_dt2(c->bl, c->stream)));
        return update(c, 1, si, si, 2, nullptr, nullptr);
    };
    auto measure = [&](double* ms) -> hweno_status {
        TRY(one());                                  // warm-up
        TRY(dev(hipStreamSynchronize(c->stream)));
        c->timer.collect();
        c->timer.reset();
        c->timer.on = true;
        c->timer.mask = (1u << hw::KC_COUNT) - 1u;
        for (int r = 0; r < reps; ++r) TRY(one());
        TRY(dev(hipStreamSynchronize(c->stream)));
        c->timer.collect();
        for (int k = 0; k < hw::KC_COUNT; ++k) ms[k] = c->timer.ms[k];
        c->timer.on = was_on;
        c->timer.mask = was_mask;
        c->timer.reset();
        return HWENO_OK;
    };
    // candidate 2 differs in the flux path (fused into the update) and in the
    // gradient kernel (weak moments formed inside it)
    const hw::Tiles cand[3] = {{16, 32, 64, 1}, {32, 64, 128, 1}, {16, 0, 0, 1}};
    double ms[3][hw::KC_COUNT];
    for (int q = 0; q < 3; ++q) {
        c->tiles = cand[q];
        TRY(upload_grids(c));
        TRY(measure(ms[q]));
    }
    // face fluxes + update: split (two flux kernels, then the update) or fused
    double fu[3];
    for (int q = 0; q < 3; ++q)
        fu[q] = ms[q][hw::KC_FLUX] + ms[q][hw::KC_UPDATE] + ms[q][hw::KC_FLUXUP];
    hw::Tiles best;
    best.recon = ms[0][hw::KC_RECON] <= ms[1][hw::KC_RECON] ? cand[0].recon : cand[1].recon;
    // weak moments + gradients: the split kernels (32 or 64 cells) or the fused one
    int gq = 0;
    for (int q = 1; q < 3; ++q)
        if (ms[q][hw::KC_RBAR] + ms[q][hw::KC_GRAD] < ms[gq][hw::KC_RBAR] + ms[gq][hw::KC_GRAD])
            gq = q;
    best.grad = cand[gq].grad;
    const int fq = fu[2] < std::min(fu[0], fu[1]) ? 2 : (fu[0] <= fu[1] ? 0 : 1);
    best.flux = cand[fq].flux;
    c->tiles = best;
    {
        // block order: XCD-aware or as launched
        double tot[2];
        for (int x = 0; x < 2; ++x) {
            c->tiles.xcd = x;
            TRY(upload_grids(c));
            double m[hw::KC_COUNT];
            TRY(measure(m));
            tot[x] = 0.0;
            for (int k = 0; k < hw::KC_COUNT; ++k) tot[x] += m[k];
        }
        c->tiles.xcd = tot[1] <= tot[0] ? 1 : 0;
    }
    if (c->batch && c->in.size() > 1) {
        // schedule order: as given vs largest instance first
        double tot[2];
        for (int o = 0; o < 2; ++o) {
            c->order_mode = o;
            TRY(upload_grids(c));
            double m[hw::KC_COUNT];
            TRY(measure(m));
            tot[o] = 0.0;
            for (int k = 0; k < hw::KC_COUNT; ++k) tot[o] += m[k];
        }
        c->order_mode = tot[1] < tot[0] ? 1 : 0;
    }
    TRY(upload_grids(c));
    if (c->batch) {
        for (auto& st : c->hst) st.active = 0;
        TRY(upload_state(c));
    }
    if (chosen) TRY(hweno_get_tiles(c, chosen));
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_set_timing(hweno_ctx* c, int enable) {
    GUARD_BEGIN
    if (!c) return HWENO_E_INVAL;
    if (enable) {
        if (!c->timer.init()) return HWENO_E_DEVICE;
        c->timer.on = true;
        c->timer.mask = (unsigned)enable & ((1u << hw::KC_COUNT) - 1u);
    } else {
        c->timer.on = false;
    }
    return HWENO_OK;
    GUARD_END
}

HWENO_API hweno_status hweno_get_timing(hweno_ctx* c, hweno_timing* out, int reset) {
    GUARD_BEGIN
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
    GUARD_END
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
        case HWENO_E_NOMEM: return "host memory allocation failed";
    }
    return "unknown status";
}

}  // extern "C"

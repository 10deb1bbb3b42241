// Host side of libsphjet: parameter validation, workspace layout, the step
// schedule (sort, two evaluations, predictor, corrector), hipGraph capture and
// the C-ABI of include/sph.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/sph.h"
#include "sph_internal.hpp"

using namespace sphjet;

static thread_local std::string g_thread_err;

namespace sphjet {

// ------------------------------------------------------------ kernel timer

hipEvent_t KernelTimer::get_() {
    if (!pool_.empty()) {
        hipEvent_t e = pool_.back();
        pool_.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

void KernelTimer::begin(const char* name, hipStream_t st) {
    if (!enabled) return;
    cur_ = name;
    cur_a_ = get_();
    (void)hipEventRecord(cur_a_, st);
}

void KernelTimer::end(hipStream_t st) {
    if (!enabled || !cur_) return;
    hipEvent_t b = get_();
    (void)hipEventRecord(b, st);
    pending_.push_back({cur_, cur_a_, b});
    cur_ = nullptr;
}

void KernelTimer::collect() {
    for (auto& p : pending_) {
        (void)hipEventSynchronize(p.b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, p.a, p.b);
        if (!total_ms.count(p.name)) names.push_back(p.name);
        total_ms[p.name] += ms;
        calls[p.name] += 1;
        pool_.push_back(p.a);
        pool_.push_back(p.b);
    }
    pending_.clear();
}

void KernelTimer::reset() {
    collect();
    names.clear();
    total_ms.clear();
    calls.clear();
}

KernelTimer::~KernelTimer() {
    for (auto& p : pending_) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool_) (void)hipEventDestroy(e);
}

}  // namespace sphjet

// ------------------------------------------------------------ workspace layout

namespace {

struct Carver {
    char* base;
    size_t off = 0;
    template <typename P>
    P* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        P* p = base ? reinterpret_cast<P*>(base + off) : nullptr;
        off += count * sizeof(P);
        return p;
    }
};

struct Grid {
    int64_t nx, ny;
    int reach;
};

const char* check_params(const sph_params& p) {
    if (!(p.h > 0) || !isfinite(p.h)) return "h must be positive";
    if (!(p.rho0 > 0)) return "rho0 must be positive";
    if (!(p.c0 > 0)) return "c0 must be positive";
    if (!(p.gamma > 0)) return "gamma must be positive";
    if (!(p.alpha >= 0)) return "alpha must be >= 0";
    if (!(p.eta2_h2 > 0)) return "eta2_h2 must be positive";
    if (!(p.sigma >= 0)) return "sigma must be >= 0";
    if (!(p.eps_h >= 0)) return "eps_h must be >= 0";
    if (!(p.courant > 0 && p.courant <= 1)) return "courant must be in (0, 1]";
    if (!(p.dt_fixed >= 0)) return "dt_fixed must be >= 0";
    if (p.kernel != SPH_WENDLAND && p.kernel != SPH_CUBIC) return "kernel must be SPH_WENDLAND or SPH_CUBIC";
    if (p.closure != 0 && p.closure != 1) return "closure must be 0 or 1";
    if (p.density != 0 && p.density != 1) return "density must be 0 or 1";
    if (p.boundary != 0 && p.boundary != 1) return "boundary must be 0 or 1";
    if (!(p.wall_spacing >= 0)) return "wall_spacing must be >= 0";
    if (!(p.box_hi[0] > p.box_lo[0] && p.box_hi[1] > p.box_lo[1])) return "box_hi must exceed box_lo";
    if (!(p.cell_size > p.h)) return "cell_size must exceed h";
    if (!isfinite(p.gravity[0]) || !isfinite(p.gravity[1])) return "gravity must be finite";
    if (p.gravity_plane != 0 && p.gravity_plane != 1) return "gravity_plane must be 0 or 1";
    if (p.gravity_plane && !(p.gravity[0] != 0.0 || p.gravity[1] != 0.0)) return "gravity_plane needs a non-zero g";
    if (p.gravity_plane && isnan(p.gravity_from)) return "gravity_from must not be NaN";
    return nullptr;
}

Grid grid_of(const sph_params& p) {
    double inv = 1.0 / p.cell_size;
    Grid g;
    g.nx = (int64_t)floor((p.box_hi[0] - p.box_lo[0]) * inv) + 1;
    g.ny = (int64_t)floor((p.box_hi[1] - p.box_lo[1]) * inv) + 1;
    g.reach = p.cell_size > 2.0 * p.h ? 1 : 2;
    return g;
}

// Bins the breakup detector may need: per system, its box's diagonal in bins of
// h/2 (the bins are half the gap, and the gap is at least h), plus a margin.
uint64_t breakup_bins(int n_sys, const sph_params* p) {
    uint64_t total = 0;
    for (int s = 0; s < n_sys; ++s)
        total += (uint64_t)ceil(hypot(p[s].box_hi[0] - p[s].box_lo[0], p[s].box_hi[1] - p[s].box_lo[1]) /
                                (0.5 * p[s].h)) + 4;
    return total;
}

// Workspace of the repulsive-force walls (systems with boundary = 1): per
// such system two grids of cells of 2h + db over its box with a margin of a
// cell, and room for a record per particle of the system.
struct WallPlan {
    uint64_t cells = 0, records = 0;
    bool any = false;
};

double wall_db(const sph_params& p) { return p.wall_spacing > 0 ? p.wall_spacing : p.h / 1.3; }

void wall_grid(const sph_params& p, double& x0, double& y0, double& cs, int32_t& nx, int32_t& ny) {
    cs = 2.0 * p.h + wall_db(p);
    x0 = p.box_lo[0] - cs;
    y0 = p.box_lo[1] - cs;
    nx = (int32_t)ceil((p.box_hi[0] - p.box_lo[0]) / cs) + 3;
    ny = (int32_t)ceil((p.box_hi[1] - p.box_lo[1]) / cs) + 3;
}

WallPlan wall_plan(int n_sys, const sph_params* p, const int64_t* off) {
    WallPlan w;
    for (int s = 0; s < n_sys; ++s) {
        if (p[s].boundary != 1) continue;
        double x0, y0, cs;
        int32_t nx, ny;
        wall_grid(p[s], x0, y0, cs, nx, ny);
        w.cells += 2ull * (uint64_t)nx * (uint64_t)ny;
        w.records += (uint64_t)(off[s + 1] - off[s]);
        w.any = true;
    }
    return w;
}

sph_options resolve(const sph_options* o) {
    sph_options r;
    memset(&r, 0, sizeof r);
    if (o) r = *o;
    if (r.dtype_bits == 0) r.dtype_bits = 32;
    if (r.block_sweep == 0) r.block_sweep = 256;
    if (r.block_stream == 0) r.block_stream = 256;
    if (r.use_graph < 0) r.use_graph = 1;
    if (r.xcd_remap < 0) r.xcd_remap = 1;
    if (r.graph_steps <= 0) r.graph_steps = 8;
    if (r.graph_steps & 1) r.graph_steps += 1;
    return r;
}

const char* check_options(const sph_options& o) {
    if (o.dtype_bits != 32 && o.dtype_bits != 64) return "dtype_bits must be 32 or 64";
    if (o.block_sweep < 64 || o.block_sweep > 256 || o.block_sweep % 64) return "block_sweep must be 64, 128, 192 or 256";
    if (o.block_stream < 64 || o.block_stream > 1024 || o.block_stream % 64) return "block_stream must be a multiple of 64 in [64, 1024]";
    return nullptr;
}

}  // namespace

// ------------------------------------------------------------ context

struct sph_ctx_base {
    virtual ~sph_ctx_base() {}
};

struct sph_ctx {
    sph_options opt;
    int n_sys = 0;
    int64_t n = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;
    std::vector<sph_params> params;
    std::vector<int64_t> offsets;
    std::vector<uint32_t> cell_base;  // n_sys + 1 (last = trash)
    KernelTimer timer;
    std::vector<std::string> prof_names;
    std::vector<const char*> prof_ptrs;
    std::unique_ptr<sph_ctx_base> impl;
    int (*step_fn)(sph_ctx*, int) = nullptr;
    int (*evaluate_fn)(sph_ctx*) = nullptr;
    int (*read_fn)(sph_ctx*, int, void*, size_t) = nullptr;
    int (*nbr_fn)(sph_ctx*, int64_t*, int32_t*, int64_t, int64_t*) = nullptr;
    int (*closure_fn)(sph_ctx*, const float*) = nullptr;
    int (*restore_fn)(sph_ctx*, const void*, size_t) = nullptr;
    int (*breakup_fn)(sph_ctx*, const double*, const double*, double, double*, int32_t*) = nullptr;
    int (*walls_fn)(sph_ctx*, const double*) = nullptr;
    int static_dev = -1;   // device whose static workspace this context holds (sph_init_static), else -1
};

// Trainer of the closure network (see sph_mlp_* in include/sph.h).
struct sph_mlp {
    hipStream_t stream = nullptr;
    int64_t max_batch = 0;
    int t = 0;
    MlpBufs B{};
    float* grad = nullptr;
    float* loss = nullptr;
    float* partial = nullptr;
    float* loss_part = nullptr;
    float* staging = nullptr;
};

static sph_status fail(sph_ctx* c, sph_status s, const std::string& msg) {
    if (c) c->err = msg;
    g_thread_err = msg;
    return s;
}

#define HIP_OK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(c, SPH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

namespace {

template <typename T>
struct Impl : sph_ctx_base {
    int n = 0, n_sys = 0;
    LaunchCfg L{};
    SysDev<T>* sys = nullptr;
    StateBuf<T> buf[2]{};
    double2* pos_h = nullptr;
    V2<T>* vel_h = nullptr;
    T* dens_h = nullptr;
    T *colour = nullptr, *drho = nullptr, *kappa = nullptr, *kappa_plain = nullptr, *aux = nullptr;
    T* vol = nullptr;
    V4<T>* eos = nullptr;
    uint4* smask = nullptr;      // skin mask (pairs within R s) of the first evaluation of a step
    uint32_t* smask4 = nullptr;
    uint32_t surf_region = 0;
    uint32_t* surf_count = nullptr;
    uint32_t* surf_list = nullptr;
    bool density_sum = false;   // some system uses the density summation (eq. 6)
    // learned closure (only when some system uses it)
    bool closure = false;
    ClosureView cl{};
    MlpBufs net{};
    V2<T>* acc = nullptr;
    V2<T>* nrm = nullptr;
    SortBufs sb{};
    unsigned long long* dtmin = nullptr;
    double* dt_wave = nullptr;
    unsigned long long* skin_max = nullptr;
    double* dt = nullptr;
    double* time = nullptr;
    uint32_t* flags = nullptr;
    int64_t* dbg_start = nullptr;
    // repulsive-force walls (some system has boundary = 1)
    bool repulsive = false;
    WallSys* wall_sys = nullptr;
    uint32_t* wall_cstart = nullptr;
    double4* wall_rec = nullptr;
    V2<T>* fwall = nullptr;
    uint64_t wall_cells = 0;
    unsigned long long* brk_sys = nullptr;    // breakup detector: per-system arrays
    unsigned long long* brk_bins = nullptr;   // and its bins (minima, then maxima)
    uint64_t brk_capacity = 0;
    int cur = 0;
    bool graphs = false;
    int graph_steps = 0;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};   // one step from buffer k
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t mexec[2] = {nullptr, nullptr};   // graph_steps steps from buffer k (back to k)
    hipGraph_t mgraph[2] = {nullptr, nullptr};

    ~Impl() override {
        for (int k = 0; k < 2; ++k) {
            if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
            if (mexec[k]) (void)hipGraphExecDestroy(mexec[k]);
            if (mgraph[k]) (void)hipGraphDestroy(mgraph[k]);
        }
    }

    // Lays out every buffer in the workspace (base == nullptr: size only).
    size_t carve(char* base, int64_t n_, int n_sys_, uint32_t trash, int block_stream, bool with_closure,
                 uint64_t bins, const WallPlan& wp) {
        Carver cv{base};
        closure = with_closure;
        if (with_closure) {
            cl.count = cv.take<uint32_t>(4);
            cl.list = cv.take<uint32_t>(n_);
            cl.stencil = cv.take<uint16_t>((size_t)64 * n_);
            cl.out = cv.take<float>((size_t)4 * n_);
            cl.fallback = cv.take<uint32_t>(n_);
            cl.capacity = (uint32_t)n_;
            net.master = cv.take<float>(MLP_NPARAMS);
            net.wt1 = cv.take<uint16_t>(64 * 64);
            net.wt2 = cv.take<uint16_t>(64 * 64);
            net.wt3 = cv.take<uint16_t>(16 * 64);
            net.w2 = cv.take<uint16_t>(64 * 64);
            net.w3 = cv.take<uint16_t>(64 * 16);
            net.b1 = cv.take<float>(64);
            net.b2 = cv.take<float>(64);
            net.b3 = cv.take<float>(16);
        }
        sys = cv.take<SysDev<T>>(n_sys_);
        for (int k = 0; k < 2; ++k) {
            buf[k].pos = cv.take<double2>(n_ + POS_PAD);
            buf[k].vel = cv.take<V2<T>>(n_);
            buf[k].dens = cv.take<T>(n_);
            buf[k].mass = cv.take<T>(n_);
            buf[k].tag = cv.take<uint32_t>(n_);
            buf[k].id = cv.take<uint32_t>(n_);
        }
        pos_h = cv.take<double2>(n_ + POS_PAD);
        vel_h = cv.take<V2<T>>(n_);
        dens_h = cv.take<T>(n_);
        colour = cv.take<T>(n_);
        drho = cv.take<T>(n_);
        acc = cv.take<V2<T>>(n_);
        nrm = cv.take<V2<T>>(n_);
        kappa = cv.take<T>(n_);
        kappa_plain = cv.take<T>(n_);
        aux = cv.take<T>(n_ < 2 ? 2 : n_);
        vol = cv.take<T>(n_);
        eos = cv.take<V4<T>>(n_);
        smask = cv.take<uint4>(n_);
        smask4 = cv.take<uint32_t>(n_);
        surf_region = (uint32_t)surface_region(n_, n_sys_);
        surf_count = cv.take<uint32_t>(SURF_REGIONS);
        sb.surf_count = surf_count;
        surf_list = cv.take<uint32_t>((size_t)SURF_REGIONS * surf_region);
        int64_t nb = (n_ + block_stream - 1) / block_stream;
        sb.trash = trash;
        sb.count = cv.take<uint32_t>((size_t)trash + 1);
        sb.cstart = cv.take<uint32_t>((size_t)trash + 2);
        sb.key = cv.take<uint32_t>(n_);
        sb.slot = cv.take<uint32_t>(n_);
        sb.blk = cv.take<uint32_t>(nb + 1);
        sb.part = cv.take<uint32_t>(scan_tiles((int64_t)trash + 1) + 1);
        sb.part2 = cv.take<uint32_t>(scan_tiles(nb) + 1);
        sb.cell_ids = cv.take<uint32_t>(n_);
        sb.scratch = cv.take<uint32_t>(n_);
        sb.cell = cv.take<uint32_t>(n_);
        sb.sys_cell_base = cv.take<uint32_t>(n_sys_ + 1);
        sb.sys_lo = cv.take<uint32_t>(n_sys_);
        sb.sys_hi = cv.take<uint32_t>(n_sys_);
        sb.chunk_base = cv.take<uint32_t>(n_sys_ + 1);
        dtmin = cv.take<unsigned long long>(2 * n_sys_);
        dt_wave = cv.take<double>(2 * surface_chunks(n_, n_sys_));
        skin_max = cv.take<unsigned long long>(n_sys_ + 1);
        dt = cv.take<double>(n_sys_);
        time = cv.take<double>(n_sys_);
        flags = cv.take<uint32_t>(4);
        dbg_start = cv.take<int64_t>(n_ + 1);
        brk_sys = cv.take<unsigned long long>((size_t)8 * n_sys_ + 2);
        brk_bins = cv.take<unsigned long long>(2 * bins);
        brk_capacity = bins;
        repulsive = wp.any;
        if (wp.any) {
            wall_sys = cv.take<WallSys>(n_sys_);
            wall_cstart = cv.take<uint32_t>(wp.cells + 1);
            wall_rec = cv.take<double4>(wp.records ? wp.records : 1);
            fwall = cv.take<V2<T>>(n_);
            wall_cells = wp.cells;
        }
        return cv.off + 256;
    }

    EvalView<T> eval_view(bool half, bool do_dt) const {
        const StateBuf<T>& S = buf[cur];
        EvalView<T> v{};
        v.n = n;
        v.xcd = L.xcd;
        v.do_dt = do_dt ? 1 : 0;
        v.n_sys = n_sys;
        v.sys_lo = sb.sys_lo;
        v.sys_hi = sb.sys_hi;
        v.chunk_base = sb.chunk_base;
        v.sys = sys;
        v.pos = half ? pos_h : S.pos;
        v.vel = half ? vel_h : S.vel;
        v.dens = half ? dens_h : S.dens;
        v.mass = S.mass;
        v.tag = S.tag;
        v.id = S.id;
        v.cell = sb.cell;
        v.cstart = sb.cstart;
        v.colour = colour;
        v.drho = drho;
        v.acc = acc;
        v.nrm = nrm;
        v.kappa = kappa;
        v.kappa_plain = kappa_plain;
        v.dtmin = dtmin;
        v.dt_wave = dt_wave;
        v.vol = vol;
        v.eos = eos;
        // the first evaluation of a step scans the cells and writes the skin
        // mask (pairs within R s); both evaluations walk it with the exact pair
        // predicate
        v.nmask = smask;
        v.nmask4 = smask4;
        v.smask = half ? nullptr : smask;
        v.smask4 = half ? nullptr : smask4;
        v.surf_region = surf_region;
        v.surf_count = surf_count;
        v.surf_list = surf_list;
        if (closure) {
            v.cl_count = cl.count;
            v.cl_list = cl.list;
            v.cl_capacity = cl.capacity;
        }
        v.skin_max = half ? skin_max : nullptr;
        v.flags = flags;
        v.dens_out = half ? dens_h : S.dens;
        v.vol_out = vol;
        v.density_sum = density_sum ? 1 : 0;
        v.fwall = fwall;
        return v;
    }

    // One evaluation of every right-hand side at the current (or half-step) state.
    void evaluate(bool half, bool do_dt, hipStream_t st, KernelTimer* kt) {
        if (closure) launch_fill_u32(cl.count, 1, 0u, st);
        EvalView<T> v = eval_view(half, do_dt);
        // the wall force runs whenever some system has repulsive walls: the step
        // graphs are captured before sph_set_wall_normals fills the grids,
        // which are empty (no force) until then
        WallView W{wall_sys, wall_cstart, wall_rec, time, dt, half ? 1 : 0, 0};
        launch_eval<T>(L, v, repulsive ? &W : nullptr, st, kt);
        if (closure) launch_closure<T>(v, cl, net.view(), cl.capacity, st, kt);
    }

    IntegView<T> integ_view() const {
        const StateBuf<T>& S = buf[cur];
        IntegView<T> v{};
        v.n = n;
        v.n_sys = n_sys;
        v.sys = sys;
        v.pos = S.pos;
        v.vel = S.vel;
        v.dens = S.dens;
        v.tag = S.tag;
        v.drho = drho;
        v.acc = acc;
        v.pos_h = pos_h;
        v.vel_h = vel_h;
        v.dens_h = dens_h;
        v.dt = dt;
        v.time = time;
        v.flags = flags;
        v.mass = S.mass;
        v.vol = vol;
        v.surf_count = surf_count;
        v.skin_max = skin_max;
        return v;
    }

    // Whether the current buffer's sort keys, slots and cell counts are
    // already written: every step's corrector writes them for the state it
    // produces, so the next sort starts at the count scan.
    bool keys_fresh = false;

    // Sort the current buffer into the other one; the other becomes current.
    void sort(hipStream_t st, KernelTimer* kt) {
        launch_sort<T>(L, sb, sys, buf[cur], buf[cur ^ 1], vol, keys_fresh, st, kt);
        keys_fresh = false;
        cur ^= 1;
    }

    // The current buffer's keys, where no corrector wrote them (after set-up,
    // a restore or a sort outside a step).
    void prepare_keys(hipStream_t st, KernelTimer* kt) {
        if (!keys_fresh) launch_key<T>(L, sb, sys, buf[cur], st, kt);
        keys_fresh = true;
    }

    // Before the state is overwritten: counts of keys that will not be
    // sorted are cleared, so the next key pass starts from zero.
    void discard_keys(hipStream_t st) {
        if (keys_fresh) launch_fill_u32(sb.count, (size_t)sb.trash + 1, 0u, st);
        keys_fresh = false;
    }

    // One predictor-corrector step, enqueued on st.
    void step(hipStream_t st, KernelTimer* kt) {
        sort(st, kt);
        evaluate(false, true, st, kt);
        launch_dt<T>(n_sys, sys, sb.chunk_base, dt_wave, dtmin, dt, skin_max, st, kt);
        launch_predict<T>(L, integ_view(), st, kt);
        evaluate(true, false, st, kt);
        IntegView<T> cv = integ_view();
        cv.key = sb.key;
        cv.kslot = sb.slot;
        cv.kcount = sb.count;
        cv.kblk = sb.blk;
        cv.trash = sb.trash;
        launch_correct<T>(L, cv, n_sys, dt, time, st, kt);
        keys_fresh = true;
    }
};

template <typename T>
Impl<T>* impl_of(sph_ctx* c) { return static_cast<Impl<T>*>(c->impl.get()); }

template <typename T>
int step_impl(sph_ctx* c, int n_steps) {
    Impl<T>* m = impl_of<T>(c);
    int left = n_steps;
    if (m->graphs) {
        // the graphs' first sort takes the keys a corrector wrote
        if (left > 0) m->prepare_keys(c->stream, &c->timer);
        while (left >= m->graph_steps) {
            HIP_OK(hipGraphLaunch(m->mexec[m->cur], c->stream));
            left -= m->graph_steps;
        }
        for (; left > 0; --left) {
            HIP_OK(hipGraphLaunch(m->gexec[m->cur], c->stream));
            m->cur ^= 1;
        }
    }
    for (; left > 0; --left) m->step(c->stream, &c->timer);
    HIP_OK(hipGetLastError());
    return SPH_OK;
}

template <typename T>
int evaluate_impl(sph_ctx* c) {
    Impl<T>* m = impl_of<T>(c);
    m->sort(c->stream, &c->timer);
    m->evaluate(false, true, c->stream, &c->timer);
    launch_dt<T>(m->n_sys, m->sys, m->sb.chunk_base, m->dt_wave, m->dtmin, m->dt, m->skin_max, c->stream,
                 &c->timer);
    HIP_OK(hipGetLastError());
    return SPH_OK;
}

template <typename T>
__global__ void k_nflag(int n, const SysDev<T>* sys, const uint32_t* tag, const V2<T>* nrm, int32_t* out) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    uint32_t t = tag[a];
    int f = 0;
    if (tag_type(t) == T_FLUID) {
        V2<T> v = nrm[a];
        f = sqrt_(v.x * v.x + v.y * v.y) > sys[tag_sys(t)].eps ? 1 : 0;
    }
    out[a] = f;
}

template <typename SRC>
void unpermute(const std::vector<uint32_t>& ids, const SRC* src, int comps, double* dst) {
    for (size_t j = 0; j < ids.size(); ++j)
        for (int k = 0; k < comps; ++k) dst[(size_t)ids[j] * comps + k] = (double)src[j * comps + k];
}

// The checkpoint blob of sph_read(SPH_F_ALL_STATE) and sph_restore: a header,
// then per system time and dt (FP64), then per particle in id order the stored
// values themselves: position (2 FP64), velocity (2 T), rho - rho0 (T), mass
// (T) and type (int32). Restoring these bits restores the state bit for bit.
struct StateHeader {
    uint32_t magic;        // 'SPHS'
    uint32_t version;
    uint32_t dtype_bits;
    uint32_t n_sys;
    uint64_t n;
};
constexpr uint32_t STATE_MAGIC = 0x53485053u;

template <typename T>
size_t state_bytes(int64_t n, int n_sys) {
    return sizeof(StateHeader) + (size_t)n_sys * 16 + (size_t)n * (16 + 2 * sizeof(T) + 2 * sizeof(T) + 4);
}

template <typename T>
int read_impl(sph_ctx* c, int field, void* host, size_t bytes) {
    Impl<T>* m = impl_of<T>(c);
    const int64_t n = m->n;
    const int ns = m->n_sys;
    const StateBuf<T>& S = m->buf[m->cur];
    hipStream_t st = c->stream;
    size_t want = 0;
    switch (field) {
        case SPH_F_POS: case SPH_F_VEL: case SPH_F_ACCEL: case SPH_F_NORMAL: want = (size_t)n * 16; break;
        case SPH_F_RHO: case SPH_F_PRESSURE: case SPH_F_MASS: case SPH_F_DRHODT: case SPH_F_COLOUR:
        case SPH_F_CURV: case SPH_F_CURV_PLAIN: case SPH_F_SORT_KEYS: case SPH_F_SORT_PERM:
            want = (size_t)n * 8; break;
        case SPH_F_TYPE: case SPH_F_NFLAG: case SPH_F_FALLBACK: want = (size_t)n * 4; break;
        case SPH_F_ALL_STATE: want = state_bytes<T>(n, ns); break;
        case SPH_F_STENCIL: want = (size_t)n * 64 * 8; break;
        case SPH_F_CLOSURE: want = (size_t)n * 4 * 8; break;
        case SPH_F_DT: case SPH_F_TIME: case SPH_F_NACTIVE: want = (size_t)ns * 8; break;
        case SPH_F_FLAGS: want = 4; break;
        default: return fail(c, SPH_EINVAL, "unknown field");
    }
    if (!host || bytes != want)
        return fail(c, SPH_EINVAL, "field " + std::to_string(field) + " needs " + std::to_string(want) + " bytes");
    std::vector<uint32_t> ids(n);
    HIP_OK(hipMemcpyAsync(ids.data(), S.id, n * 4, hipMemcpyDeviceToHost, st));
    double* out = static_cast<double*>(host);
    auto fetch = [&](const void* dev, size_t sz, std::vector<char>& tmp) -> hipError_t {
        tmp.resize(sz);
        hipError_t e = hipMemcpyAsync(tmp.data(), dev, sz, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(st);
    };
    std::vector<char> tmp;
    switch (field) {
        case SPH_F_POS:
            HIP_OK(fetch(S.pos, n * 16, tmp));
            unpermute(ids, reinterpret_cast<const double*>(tmp.data()), 2, out);
            break;
        case SPH_F_VEL:
            HIP_OK(fetch(S.vel, n * sizeof(V2<T>), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 2, out);
            break;
        case SPH_F_ACCEL:
            HIP_OK(fetch(m->acc, n * sizeof(V2<T>), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 2, out);
            break;
        case SPH_F_NORMAL:
            HIP_OK(fetch(m->nrm, n * sizeof(V2<T>), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 2, out);
            break;
        case SPH_F_RHO: {
            HIP_OK(fetch(S.dens, n * sizeof(T), tmp));
            std::vector<char> tg;
            HIP_OK(fetch(S.tag, n * 4, tg));
            const T* d = reinterpret_cast<const T*>(tmp.data());
            const uint32_t* tgs = reinterpret_cast<const uint32_t*>(tg.data());
            for (int64_t j = 0; j < n; ++j) out[ids[j]] = c->params[tgs[j] >> 4].rho0 + (double)d[j];
            break;
        }
        case SPH_F_PRESSURE:
            launch_pressure<T>((int)n, m->sys, S.tag, S.dens, m->aux, st);
            HIP_OK(fetch(m->aux, n * sizeof(T), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 1, out);
            break;
        case SPH_F_MASS:
            HIP_OK(fetch(S.mass, n * sizeof(T), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 1, out);
            break;
        case SPH_F_DRHODT:
            HIP_OK(fetch(m->drho, n * sizeof(T), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 1, out);
            break;
        case SPH_F_COLOUR:
            HIP_OK(fetch(m->colour, n * sizeof(T), tmp));
            unpermute(ids, reinterpret_cast<const T*>(tmp.data()), 1, out);
            break;
        case SPH_F_CURV:
        case SPH_F_CURV_PLAIN: {
            // the curvature arrays hold values for particles that pass the
            // normal filter only; every other particle reads 0
            int32_t* dev = reinterpret_cast<int32_t*>(m->aux);
            k_nflag<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>((int)n, m->sys, S.tag, m->nrm, dev);
            std::vector<char> fl;
            HIP_OK(fetch(dev, n * 4, fl));
            HIP_OK(fetch(field == SPH_F_CURV ? m->kappa : m->kappa_plain, n * sizeof(T), tmp));
            T* kv = reinterpret_cast<T*>(tmp.data());
            const int32_t* f = reinterpret_cast<const int32_t*>(fl.data());
            for (int64_t j = 0; j < n; ++j)
                if (!f[j]) kv[j] = T(0);
            unpermute(ids, kv, 1, out);
            break;
        }
        case SPH_F_TYPE: {
            HIP_OK(fetch(S.tag, n * 4, tmp));
            const uint32_t* tg = reinterpret_cast<const uint32_t*>(tmp.data());
            int32_t* o = static_cast<int32_t*>(host);
            for (int64_t j = 0; j < n; ++j) o[ids[j]] = (int32_t)(tg[j] & 15u);
            break;
        }
        case SPH_F_NFLAG: {
            int32_t* dev = reinterpret_cast<int32_t*>(m->aux);
            k_nflag<T><<<(unsigned)((n + 255) / 256), 256, 0, st>>>((int)n, m->sys, S.tag, m->nrm, dev);
            HIP_OK(fetch(dev, n * 4, tmp));
            const int32_t* f = reinterpret_cast<const int32_t*>(tmp.data());
            int32_t* o = static_cast<int32_t*>(host);
            for (int64_t j = 0; j < n; ++j) o[ids[j]] = f[j];
            break;
        }
        case SPH_F_SORT_KEYS: {
            HIP_OK(fetch(m->sb.cell, n * 4, tmp));
            const uint32_t* k = reinterpret_cast<const uint32_t*>(tmp.data());
            uint64_t* o = static_cast<uint64_t*>(host);
            for (int64_t j = 0; j < n; ++j) o[j] = k[j];
            break;
        }
        case SPH_F_SORT_PERM: {
            HIP_OK(hipStreamSynchronize(st));
            int64_t* o = static_cast<int64_t*>(host);
            for (int64_t j = 0; j < n; ++j) o[j] = ids[j];
            break;
        }
        case SPH_F_DT:
            HIP_OK(fetch(m->dt, ns * 8, tmp));
            memcpy(host, tmp.data(), ns * 8);
            break;
        case SPH_F_TIME:
            HIP_OK(fetch(m->time, ns * 8, tmp));
            memcpy(host, tmp.data(), ns * 8);
            break;
        case SPH_F_NACTIVE: {
            std::vector<uint32_t> starts(ns + 1);
            for (int s = 0; s <= ns; ++s)
                HIP_OK(hipMemcpyAsync(&starts[s], m->sb.cstart + c->cell_base[s], 4, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            int64_t* o = static_cast<int64_t*>(host);
            for (int s = 0; s < ns; ++s) o[s] = (int64_t)starts[s + 1] - (int64_t)starts[s];
            break;
        }
        case SPH_F_FLAGS:
            HIP_OK(fetch(m->flags, 4, tmp));
            memcpy(host, tmp.data(), 4);
            break;
        case SPH_F_ALL_STATE: {
            char* o = static_cast<char*>(host);
            StateHeader hd{STATE_MAGIC, 1u, (uint32_t)(8 * sizeof(T)), (uint32_t)ns, (uint64_t)n};
            memcpy(o, &hd, sizeof hd);
            o += sizeof hd;
            HIP_OK(fetch(m->time, ns * 8, tmp));
            memcpy(o, tmp.data(), ns * 8);
            o += ns * 8;
            HIP_OK(fetch(m->dt, ns * 8, tmp));
            memcpy(o, tmp.data(), ns * 8);
            o += ns * 8;
            // each per-slot array moved to id order as raw bytes
            auto raw = [&](const void* dev, size_t elem) -> hipError_t {
                hipError_t e = fetch(dev, (size_t)n * elem, tmp);
                if (e != hipSuccess) return e;
                for (int64_t j = 0; j < n; ++j) memcpy(o + (size_t)ids[j] * elem, tmp.data() + (size_t)j * elem, elem);
                o += (size_t)n * elem;
                return hipSuccess;
            };
            HIP_OK(raw(S.pos, 16));
            HIP_OK(raw(S.vel, 2 * sizeof(T)));
            HIP_OK(raw(S.dens, sizeof(T)));
            HIP_OK(raw(S.mass, sizeof(T)));
            HIP_OK(fetch(S.tag, n * 4, tmp));
            const uint32_t* tg = reinterpret_cast<const uint32_t*>(tmp.data());
            for (int64_t j = 0; j < n; ++j) {
                const int32_t ty = (int32_t)(tg[j] & 15u);
                memcpy(o + (size_t)ids[j] * 4, &ty, 4);
            }
            break;
        }
        case SPH_F_STENCIL: case SPH_F_CLOSURE: case SPH_F_FALLBACK: {
            memset(host, 0, bytes);
            if (!m->closure) break;
            uint32_t cnt = 0;
            HIP_OK(hipMemcpyAsync(&cnt, m->cl.count, 4, hipMemcpyDeviceToHost, st));
            HIP_OK(hipStreamSynchronize(st));
            if (cnt > m->cl.capacity) cnt = m->cl.capacity;
            if (field == SPH_F_FALLBACK) {
                HIP_OK(fetch(m->cl.fallback, n * 4, tmp));
                const uint32_t* f = reinterpret_cast<const uint32_t*>(tmp.data());
                std::vector<uint32_t> lst(cnt);
                if (cnt) HIP_OK(hipMemcpyAsync(lst.data(), m->cl.list, cnt * 4, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                int32_t* o = static_cast<int32_t*>(host);
                for (uint32_t k = 0; k < cnt; ++k) o[ids[lst[k]]] = (int32_t)f[lst[k]];
                break;
            }
            std::vector<uint32_t> lst(cnt);
            if (cnt) HIP_OK(hipMemcpyAsync(lst.data(), m->cl.list, cnt * 4, hipMemcpyDeviceToHost, st));
            if (field == SPH_F_STENCIL) {
                std::vector<uint16_t> rows((size_t)cnt * 64);
                if (cnt) HIP_OK(hipMemcpyAsync(rows.data(), m->cl.stencil, rows.size() * 2, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                for (uint32_t k = 0; k < cnt; ++k)
                    for (int j = 0; j < 64; ++j) {
                        uint32_t u = (uint32_t)rows[(size_t)k * 64 + j] << 16;
                        float f;
                        memcpy(&f, &u, 4);
                        out[(size_t)ids[lst[k]] * 64 + j] = (double)f;
                    }
            } else {
                std::vector<float> rows((size_t)cnt * 4);
                if (cnt) HIP_OK(hipMemcpyAsync(rows.data(), m->cl.out, rows.size() * 4, hipMemcpyDeviceToHost, st));
                HIP_OK(hipStreamSynchronize(st));
                for (uint32_t k = 0; k < cnt; ++k)
                    for (int j = 0; j < 4; ++j) out[(size_t)ids[lst[k]] * 4 + j] = j < 3 ? rows[(size_t)k * 4 + j] : 1.0;
            }
            break;
        }
    }
    uint32_t fl = 0;
    HIP_OK(hipMemcpyAsync(&fl, m->flags, 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    if (fl & ~FLAG_RESCAN) return fail(c, SPH_EUNSTABLE, "instability flags " + std::to_string(fl));
    return SPH_OK;
}

template <typename T>
int nbr_impl(sph_ctx* c, int64_t* start, int32_t* nbr, int64_t cap, int64_t* total) {
    Impl<T>* m = impl_of<T>(c);
    const int n = m->n;
    hipStream_t st = c->stream;
    // the current state sorted, and the skin mask the sweeps walk recorded
    m->sort(st, &c->timer);
    launch_colour_mask<T>(m->L, m->eval_view(false, false), st);
    EvalView<T> v = m->eval_view(false, false);
    uint32_t* cnt = m->sb.scratch;
    launch_nbr_count<T>(m->L, v, cnt, st);
    std::vector<uint32_t> counts(n), ids(n);
    HIP_OK(hipMemcpyAsync(counts.data(), cnt, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(ids.data(), m->buf[m->cur].id, (size_t)n * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    std::vector<int64_t> sstart(n + 1, 0);
    for (int j = 0; j < n; ++j) sstart[j + 1] = sstart[j] + counts[j];
    int64_t tot = sstart[n];
    // id-order start
    std::vector<int64_t> idcount(n, 0);
    for (int j = 0; j < n; ++j) idcount[ids[j]] = counts[j];
    start[0] = 0;
    for (int a = 0; a < n; ++a) start[a + 1] = start[a] + idcount[a];
    *total = tot;
    if (cap < tot || !nbr) return fail(c, SPH_ECAPACITY, "neighbour buffer too small");
    HIP_OK(hipMemcpyAsync(m->dbg_start, sstart.data(), (size_t)(n + 1) * 8, hipMemcpyHostToDevice, st));
    // fill in chunks through the half-step buffers (idle between steps)
    uint32_t* chunk = reinterpret_cast<uint32_t*>(m->pos_h);
    const int64_t chunk_cap = (int64_t)n * 4;   // 16 bytes per particle of pos_h
    std::vector<uint32_t> host_chunk;
    int a0 = 0;
    while (a0 < n) {
        int a1 = a0;
        while (a1 < n && sstart[a1 + 1] - sstart[a0] <= chunk_cap) ++a1;
        if (a1 == a0) return fail(c, SPH_ECAPACITY, "a particle has too many neighbours");
        launch_nbr_fill<T>(v, a0, a1, m->dbg_start, sstart[a0], chunk, st);
        int64_t len = sstart[a1] - sstart[a0];
        host_chunk.resize((size_t)len);
        if (len) HIP_OK(hipMemcpyAsync(host_chunk.data(), chunk, (size_t)len * 4, hipMemcpyDeviceToHost, st));
        HIP_OK(hipStreamSynchronize(st));
        for (int j = a0; j < a1; ++j) {
            int64_t o = start[ids[j]];
            int64_t cnt_j = sstart[j + 1] - sstart[j];
            for (int64_t k = 0; k < cnt_j; ++k) nbr[o + k] = (int32_t)host_chunk[(size_t)(sstart[j] - sstart[a0] + k)];
            std::sort(nbr + o, nbr + o + cnt_j);
        }
        a0 = a1;
    }
    return SPH_OK;
}

template <typename T>
int closure_impl(sph_ctx* c, const float* params) {
    Impl<T>* m = impl_of<T>(c);
    if (!m->closure) return fail(c, SPH_ESTATE, "no system of this context uses the closure");
    HIP_OK(hipMemcpyAsync(m->net.master, params, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, c->stream));
    launch_mlp_set(m->net, m->net.master, c->stream);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

template <typename T>
int restore_impl(sph_ctx* c, const void* blob, size_t bytes) {
    Impl<T>* m = impl_of<T>(c);
    const int64_t n = m->n;
    const int ns = m->n_sys;
    if (bytes != state_bytes<T>(n, ns))
        return fail(c, SPH_EINVAL, "state blob needs " + std::to_string(state_bytes<T>(n, ns)) + " bytes");
    const char* in = static_cast<const char*>(blob);
    StateHeader hd;
    memcpy(&hd, in, sizeof hd);
    if (hd.magic != STATE_MAGIC || hd.version != 1u)
        return fail(c, SPH_EINVAL, "not a state blob of this library");
    if (hd.dtype_bits != 8 * sizeof(T) || hd.n_sys != (uint32_t)ns || hd.n != (uint64_t)n)
        return fail(c, SPH_EINVAL, "state blob of another shape (dtype, systems or particle count)");
    in += sizeof hd;
    const double* time = reinterpret_cast<const double*>(in);
    const double* dt = time + ns;
    in += (size_t)ns * 16;
    const char* pos = in;
    const char* vel = pos + (size_t)n * 16;
    const char* dens = vel + (size_t)n * 2 * sizeof(T);
    const char* mass = dens + (size_t)n * sizeof(T);
    const char* type = mass + (size_t)n * sizeof(T);
    std::vector<uint32_t> tag(n), id(n);
    for (int s = 0; s < ns; ++s) {
        if (!(time[s] >= 0.0) || !(dt[s] >= 0.0)) return fail(c, SPH_EINVAL, "state blob holds a bad time or dt");
        for (int64_t a = c->offsets[s]; a < c->offsets[s + 1]; ++a) {
            int32_t ty;
            memcpy(&ty, type + (size_t)a * 4, 4);
            if (ty < SPH_FLUID || ty > SPH_INACTIVE)
                return fail(c, SPH_EINVAL, "particle type out of range at id " + std::to_string(a));
            tag[a] = ((uint32_t)s << 4) | (uint32_t)ty;
            id[a] = (uint32_t)a;
        }
    }
    hipStream_t st = c->stream;
    HIP_OK(hipStreamSynchronize(st));
    m->discard_keys(st);   // the keys of the state being replaced
    // the blob's arrays are in id order: slot a holds particle a until the sort
    StateBuf<T>& X = m->buf[m->cur];
    HIP_OK(hipMemcpyAsync(X.pos, pos, (size_t)n * 16, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.vel, vel, (size_t)n * 2 * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.dens, dens, (size_t)n * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.mass, mass, (size_t)n * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.tag, tag.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.id, id.data(), (size_t)n * 4, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(m->time, time, (size_t)ns * 8, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(m->dt, dt, (size_t)ns * 8, hipMemcpyHostToDevice, st));
    // derived fields belong to the state they were evaluated at: cleared
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->colour), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->drho), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->acc), n * sizeof(V2<T>) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->nrm), n * sizeof(V2<T>) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->kappa), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->kappa_plain), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(m->flags, 4, 0u, st);
    m->sort(st, &c->timer);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    return SPH_OK;
}

// The repulsive-force walls' grids from the boundary particles' current
// positions (pistons at their travel now) and the caller's normals.
template <typename T>
int walls_impl(sph_ctx* c, const double* normals) {
    Impl<T>* m = impl_of<T>(c);
    if (!m->repulsive) return fail(c, SPH_ESTATE, "no system of this context has repulsive-force walls");
    const int64_t n = m->n;
    const int ns = m->n_sys;
    hipStream_t st = c->stream;
    const StateBuf<T>& S = m->buf[m->cur];
    std::vector<uint32_t> ids(n), tags(n);
    std::vector<double2> pos(n);
    std::vector<double> time(ns);
    HIP_OK(hipMemcpyAsync(ids.data(), S.id, n * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(tags.data(), S.tag, n * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(pos.data(), S.pos, n * 16, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(time.data(), m->time, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    std::vector<WallSys> ws(ns);
    std::vector<uint32_t> cstart(m->wall_cells + 1, 0);
    std::vector<double4> rec;
    uint32_t cell_off = 0;
    // slots of every system's boundary particles with a normal, by grid
    std::vector<std::vector<uint32_t>> members(2 * ns);
    for (int64_t j = 0; j < n; ++j) {
        const uint32_t ty = tags[j] & 15u, s = tags[j] >> 4;
        if ((ty != SPH_WALL && ty != SPH_PISTON) || c->params[s].boundary != 1) continue;
        const double nx = normals[2 * (size_t)ids[j]], ny = normals[2 * (size_t)ids[j] + 1];
        if (nx == 0.0 && ny == 0.0) continue;
        if (!isfinite(nx) || !isfinite(ny) || fabs(nx * nx + ny * ny - 1.0) > 1e-6)
            return fail(c, SPH_EINVAL, "wall normal of particle " + std::to_string(ids[j]) + " is not a unit vector");
        members[2 * s + (ty == SPH_PISTON ? 1 : 0)].push_back((uint32_t)j);
    }
    for (int s = 0; s < ns; ++s) {
        const sph_params& p = c->params[s];
        WallSys& G = ws[s];
        memset(&G, 0, sizeof G);
        if (p.boundary != 1) continue;
        double cs;
        wall_grid(p, G.x0, G.y0, cs, G.nx, G.ny);
        G.inv_cs = 1.0 / cs;
        G.db = wall_db(p);
        const double tm = time[s];
        G.x_ref = p.piston_omega == 0.0 ? p.piston_u * tm
                                         : p.piston_u * (tm + p.piston_amp * (1.0 - cos(p.piston_omega * tm)) / p.piston_omega);
        const uint32_t cells = (uint32_t)G.nx * (uint32_t)G.ny;
        for (int g = 0; g < 2; ++g) {
            G.cell_base[g] = cell_off;
            // counting sort of the grid's records by cell
            std::vector<uint32_t> cell_of;
            for (uint32_t j : members[2 * s + g]) {
                int cx = (int)floor((pos[j].x - G.x0) * G.inv_cs), cy = (int)floor((pos[j].y - G.y0) * G.inv_cs);
                cx = std::min(std::max(cx, 0), G.nx - 1);
                cy = std::min(std::max(cy, 0), G.ny - 1);
                cell_of.push_back((uint32_t)cx * (uint32_t)G.ny + (uint32_t)cy);
            }
            std::vector<uint32_t> count(cells + 1, 0);
            for (uint32_t k : cell_of) ++count[k + 1];
            for (uint32_t k = 0; k < cells; ++k) count[k + 1] += count[k];
            const uint32_t r0 = (uint32_t)rec.size();
            rec.resize(rec.size() + cell_of.size());
            std::vector<uint32_t> fillp(count.begin(), count.end() - 1);
            for (size_t i = 0; i < cell_of.size(); ++i) {
                const uint32_t j = members[2 * s + g][i];
                double4 r;
                r.x = pos[j].x;
                r.y = pos[j].y;
                r.z = normals[2 * (size_t)ids[j]];
                r.w = normals[2 * (size_t)ids[j] + 1];
                rec[r0 + fillp[cell_of[i]]++] = r;
            }
            for (uint32_t k = 0; k <= cells; ++k) cstart[cell_off + k] = r0 + count[k];
            cell_off += cells;
        }
    }
    HIP_OK(hipMemcpyAsync(m->wall_sys, ws.data(), ns * sizeof(WallSys), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(m->wall_cstart, cstart.data(), cstart.size() * 4, hipMemcpyHostToDevice, st));
    if (!rec.empty()) HIP_OK(hipMemcpyAsync(m->wall_rec, rec.data(), rec.size() * sizeof(double4), hipMemcpyHostToDevice, st));
    HIP_OK(hipStreamSynchronize(st));
    return SPH_OK;
}

// Host twin of the order-preserving map of FP64 values to 64-bit integers.
static double from_ordered_host(unsigned long long k) {
    const unsigned long long u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    double x;
    memcpy(&x, &u, 8);
    return x;
}

template <typename T>
int breakup_impl(sph_ctx* c, const double* axis, const double* xi_start, double gap_h, double* length,
                 int32_t* broken) {
    Impl<T>* m = impl_of<T>(c);
    const int64_t n = m->n;
    const int ns = m->n_sys;
    unsigned long long* extent = m->brk_sys;
    double* start = reinterpret_cast<double*>(extent + ns);
    double* anchor = start + ns;
    double* half_gap = anchor + ns;
    double* gap = half_gap + ns;
    double* len = gap + ns;
    int32_t* brk = reinterpret_cast<int32_t*>(len + ns);
    uint32_t* base = reinterpret_cast<uint32_t*>(brk + ns + (ns & 1));
    // bins start at the nozzle exit or at the near edge of the box, whichever
    // is farther along the axis: active fluid lies inside the box
    std::vector<double> hs(xi_start, xi_start + ns), ha(ns), hg(ns), hh(ns);
    for (int s = 0; s < ns; ++s) {
        if (!isfinite(hs[s])) return fail(c, SPH_EINVAL, "xi_start must be finite");
        const sph_params& q = c->params[s];
        const double x0 = axis[0] >= 0 ? q.box_lo[0] : q.box_hi[0], y0 = axis[1] >= 0 ? q.box_lo[1] : q.box_hi[1];
        ha[s] = std::max(hs[s], x0 * axis[0] + y0 * axis[1]);
        hg[s] = gap_h * q.h;
        hh[s] = 0.5 * hg[s];
    }
    hipStream_t st = c->stream;
    const StateBuf<T>& S = m->buf[m->cur];
    HIP_OK(hipMemcpyAsync(start, hs.data(), ns * 8, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(anchor, ha.data(), ns * 8, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(gap, hg.data(), ns * 8, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(half_gap, hh.data(), ns * 8, hipMemcpyHostToDevice, st));
    launch_breakup((int)n, ns, S.tag, S.pos, axis[0], axis[1], start, extent, st);
    std::vector<unsigned long long> ext(ns);
    HIP_OK(hipMemcpyAsync(ext.data(), extent, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    // bins of half the gap from each anchor to the system's farthest particle
    std::vector<uint32_t> hb(ns + 1);
    uint64_t total = 0;
    for (int s = 0; s < ns; ++s) {
        hb[s] = (uint32_t)total;
        if (ext[s]) {
            const double u = floor((from_ordered_host(ext[s]) - ha[s]) / hh[s]);
            total += (u > 0.0 ? (uint64_t)u : 0ull) + 2;
        }
        if (total > m->brk_capacity)
            return fail(c, SPH_ECAPACITY, "fluid beyond its box along the axis: more breakup bins than the workspace holds");
    }
    hb[ns] = (uint32_t)total;
    HIP_OK(hipMemcpyAsync(base, hb.data(), (ns + 1) * 4, hipMemcpyHostToDevice, st));
    launch_breakup_bins((int)n, ns, S.tag, S.pos, axis[0], axis[1], start, anchor, half_gap, gap, base,
                        (uint32_t)total, m->brk_bins, m->brk_bins + total, len, brk, st);
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(length, len, ns * 8, hipMemcpyDeviceToHost, st));
    HIP_OK(hipMemcpyAsync(broken, brk, ns * 4, hipMemcpyDeviceToHost, st));
    HIP_OK(hipStreamSynchronize(st));
    return SPH_OK;
}

template <typename T>
SysDev<T> make_sysdev(const sph_params& p, uint32_t base) {
    SysDev<T> s;
    memset(&s, 0, sizeof s);
    Grid g = grid_of(p);
    const double PI = 3.14159265358979323846;
    s.x0 = p.box_lo[0];
    s.y0 = p.box_lo[1];
    s.inv_s = 1.0 / p.cell_size;
    s.R2 = (2.0 * p.h) * (2.0 * p.h);
    // FP32 band of the pair predicate: 2^-19 of (2h)^2 either side, rounded outwards
    s.r2_in = std::nextafter((float)(s.R2 * (1.0 - 0x1p-19)), 0.0f);
    s.r2_out = std::nextafter((float)(s.R2 * (1.0 + 0x1p-19)), INFINITY);
    double skin = g.reach * p.cell_size - 2.0 * p.h;
    s.skin2 = 0.25 * skin * skin;
    s.cell_s = p.cell_size;
    // pairs within 2h after a half step of at most skin/2 per particle were
    // within R s = 2h + skin before it (the margin covers rounding)
    s.Rs2 = (g.reach * p.cell_size) * (g.reach * p.cell_size) * (1.0 + 1e-12);
    s.nx = (int32_t)g.nx;
    s.ny = (int32_t)g.ny;
    s.reach = g.reach;
    s.kernel = p.kernel;
    s.cell_base = base;
    double h = p.h;
    double wn = p.kernel == SPH_WENDLAND ? 7.0 / (4.0 * PI * h * h) : 10.0 / (7.0 * PI * h * h);
    double gn = p.kernel == SPH_WENDLAND ? -5.0 * wn / (h * h) : wn / (h * h);
    s.h = (T)h;
    s.inv_h = (T)(1.0 / h);
    s.wnorm = (T)wn;
    s.gnorm = (T)gn;
    s.W0 = (T)wn;
    s.rho0 = (T)p.rho0;
    s.inv_rho0 = (T)(1.0 / p.rho0);
    s.B = (T)(p.rho0 * p.c0 * p.c0 / p.gamma);
    s.c0 = (T)p.c0;
    s.gamma = (T)p.gamma;
    s.half_gm1 = (T)(0.5 * (p.gamma - 1.0));
    s.alpha_h = (T)(p.alpha * h);
    s.visc_c0 = (T)(-p.alpha * h * p.c0);
    s.eta2 = (T)(p.eta2_h2 * h * h);
    s.sigma = (T)p.sigma;
    s.eps = (T)(p.eps_h / h);
    s.gx = (T)p.gravity[0];
    s.gy = (T)p.gravity[1];
    s.gamma7 = p.gamma == 7.0 ? 1 : 0;
    s.closure = p.closure;
    s.density_sum = p.density;
    s.g_plane = p.gravity_plane;
    if (p.gravity_plane) {
        const double gn = hypot(p.gravity[0], p.gravity[1]);
        s.ghx = p.gravity[0] / gn;
        s.ghy = p.gravity[1] / gn;
        s.g_from = p.gravity_from;
    }
    s.boundary = p.boundary;
    s.h64 = h;
    s.wnorm64 = wn;
    s.rho0_64 = p.rho0;
    s.closure_tol = (T)(p.closure_tol > 0 ? p.closure_tol : 0.2);
    s.courant = p.courant;
    s.dt_fixed = p.dt_fixed;
    s.box_lo_x = p.box_lo[0];
    s.box_lo_y = p.box_lo[1];
    s.box_hi_x = p.box_hi[0];
    s.box_hi_y = p.box_hi[1];
    double pn = hypot(p.piston_dir[0], p.piston_dir[1]);
    s.pdx = pn > 0 ? p.piston_dir[0] / pn : 0.0;
    s.pdy = pn > 0 ? p.piston_dir[1] / pn : 0.0;
    s.pu = p.piston_u;
    s.pamp = p.piston_amp;
    s.pomega = p.piston_omega;
    return s;
}

// Validates systems and computes cell bases; returns an error message or null.
const char* plan(const sph_options& o, int n_sys, const sph_params* p, const int64_t* off,
                 std::vector<uint32_t>& base) {
    if (const char* e = check_options(o)) return e;
    if (n_sys < 1 || n_sys >= (1 << 27)) return "n_sys must be in [1, 2^27)";
    if (!p || !off) return "params and offsets must not be NULL";
    if (off[0] != 0) return "offsets[0] must be 0";
    for (int s = 0; s < n_sys; ++s)
        if (off[s + 1] < off[s]) return "offsets must be non-decreasing";
    if (off[n_sys] < 1 || off[n_sys] > SPH_MAX_PARTICLES) return "particle count must be in [1, SPH_MAX_PARTICLES]";
    base.assign(n_sys + 1, 0);
    uint64_t acc = 0;
    for (int s = 0; s < n_sys; ++s) {
        if (const char* e = check_params(p[s])) return e;
        Grid g = grid_of(p[s]);
        if (g.nx < 1 || g.ny < 1 || g.nx > (1 << 30) || g.ny > (1 << 30)) return "cell grid out of range";
        base[s] = (uint32_t)acc;
        acc += (uint64_t)g.nx * (uint64_t)g.ny;
        if (acc > ((uint64_t)1 << 31)) return "too many cells (box / cell_size too large)";
    }
    base[n_sys] = (uint32_t)acc;
    return nullptr;
}

template <typename T>
int init_impl(sph_ctx* c, const double* pos, const double* vel, const double* rho, const double* mass,
              const int32_t* type, void* ws, size_t ws_bytes) {
    auto* m = new Impl<T>();
    c->impl.reset(m);
    m->n = (int)c->n;
    m->n_sys = c->n_sys;
    m->L.n = m->n;
    m->L.n_sys = m->n_sys;
    m->L.block_sweep = c->opt.block_sweep;
    m->L.block_stream = c->opt.block_stream;
    m->L.xcd = c->opt.xcd_remap;
    const uint32_t trash = c->cell_base[c->n_sys];
    bool with_closure = false;
    for (int s2 = 0; s2 < c->n_sys; ++s2) {
        with_closure = with_closure || c->params[s2].closure != 0;
        m->density_sum = m->density_sum || c->params[s2].density != 0;
    }
    const uint64_t bins = breakup_bins(c->n_sys, c->params.data());
    const WallPlan wp = wall_plan(c->n_sys, c->params.data(), c->offsets.data());
    size_t need = m->carve(nullptr, c->n, c->n_sys, trash, c->opt.block_stream, with_closure, bins, wp);
    if (ws_bytes < need)
        return fail(c, SPH_ENOMEM, "workspace needs " + std::to_string(need) + " bytes");
    if (((uintptr_t)ws) & 255) return fail(c, SPH_EINVAL, "workspace must be 256-byte aligned");
    m->carve(static_cast<char*>(ws), c->n, c->n_sys, trash, c->opt.block_stream, with_closure, bins, wp);
    if (with_closure) {
        // the stencil kernel builds four stencils per wave once two per wave
        // would more than fill the chip's wave slots (8 per SIMD, 4 SIMDs per CU)
        int dev = 0, ncu = 0;
        HIP_OK(hipGetDevice(&dev));
        HIP_OK(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
        m->cl.quad_min = 2u * 32u * (uint32_t)ncu;
    }
    const int64_t n = c->n;
    hipStream_t st = c->stream;
    // host staging in device format
    std::vector<SysDev<T>> sd(c->n_sys);
    for (int s = 0; s < c->n_sys; ++s) sd[s] = make_sysdev<T>(c->params[s], c->cell_base[s]);
    std::vector<double2> hp(n);
    std::vector<V2<T>> hv(n);
    std::vector<T> hd(n), hm(n);
    std::vector<uint32_t> ht(n), hi(n);
    for (int s = 0; s < c->n_sys; ++s) {
        for (int64_t a = c->offsets[s]; a < c->offsets[s + 1]; ++a) {
            if (type[a] < SPH_FLUID || type[a] > SPH_INACTIVE)
                return fail(c, SPH_EINVAL, "particle type out of range at id " + std::to_string(a));
            if (!isfinite(pos[2 * a]) || !isfinite(pos[2 * a + 1]) || !isfinite(rho[a]) || !(mass[a] > 0))
                return fail(c, SPH_EINVAL, "non-finite position/density or non-positive mass at id " + std::to_string(a));
            hp[a].x = pos[2 * a];
            hp[a].y = pos[2 * a + 1];
            hv[a].x = (T)vel[2 * a];
            hv[a].y = (T)vel[2 * a + 1];
            hd[a] = (T)(rho[a] - c->params[s].rho0);
            hm[a] = (T)mass[a];
            ht[a] = ((uint32_t)s << 4) | (uint32_t)type[a];
            hi[a] = (uint32_t)a;
        }
    }
    StateBuf<T>& X = m->buf[0];
    HIP_OK(hipMemcpyAsync(m->sys, sd.data(), sizeof(SysDev<T>) * c->n_sys, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(m->sb.sys_cell_base, c->cell_base.data(), 4 * (c->n_sys + 1), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.pos, hp.data(), n * sizeof(double2), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.vel, hv.data(), n * sizeof(V2<T>), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.dens, hd.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.mass, hm.data(), n * sizeof(T), hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.tag, ht.data(), n * 4, hipMemcpyHostToDevice, st));
    HIP_OK(hipMemcpyAsync(X.id, hi.data(), n * 4, hipMemcpyHostToDevice, st));
    // derived arrays start at zero; dt minima at +inf; time 0; flags 0
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->colour), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->drho), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->acc), n * sizeof(V2<T>) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->nrm), n * sizeof(V2<T>) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->kappa), n * sizeof(T) / 4, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(m->kappa_plain), n * sizeof(T) / 4, 0u, st);
    launch_fill_u64(m->dtmin, 2 * c->n_sys, (unsigned long long)0x7ff0000000000000ull, st);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(m->dt), c->n_sys, 0ull, st);
    launch_fill_u64(reinterpret_cast<unsigned long long*>(m->time), c->n_sys, 0ull, st);
    launch_fill_u32(m->flags, 4, 0u, st);
    launch_fill_u64(m->skin_max, c->n_sys + 1, 0ull, st);
    if (m->repulsive) {   // no wall records until sph_set_wall_normals
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->fwall), n * sizeof(V2<T>) / 4, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->wall_sys), c->n_sys * sizeof(WallSys) / 4, 0u, st);
        launch_fill_u32(m->wall_cstart, m->wall_cells + 1, 0u, st);
    }
    launch_fill_u32(m->sb.cell, n, 0u, st);
    // the padding past the last position is read (and ignored) by the candidate scan
    for (double2* p : {m->buf[0].pos, m->buf[1].pos, m->pos_h})
        launch_fill_u32(reinterpret_cast<uint32_t*>(p + n), (size_t)POS_PAD * 4, 0u, st);
    launch_fill_u32(m->sb.count, (size_t)m->sb.trash + 1, 0u, st);   // kept zero between sorts
    if (m->closure) {
        launch_fill_u32(m->cl.count, 4, 0u, st);
        launch_fill_u32(m->cl.fallback, n, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->cl.stencil), (size_t)32 * n, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->cl.out), (size_t)4 * n, 0u, st);
        std::vector<float> zeros(MLP_NPARAMS, 0.f);
        HIP_OK(hipMemcpyAsync(m->net.master, zeros.data(), sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, st));
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->net.wt3), 16 * 64 / 2, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->net.w3), 64 * 16 / 2, 0u, st);
        launch_fill_u32(reinterpret_cast<uint32_t*>(m->net.b3), 16, 0u, st);
        launch_mlp_set(m->net, m->net.master, st);
        HIP_OK(hipStreamSynchronize(st));
    }
    // a first sort so the state is cell-ordered from the start
    m->sort(st, &c->timer);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    if (c->opt.use_graph) {
        HIP_OK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        int saved = m->cur;
        const bool saved_keys = m->keys_fresh;
        m->keys_fresh = true;   // replays start from keys written by a corrector (step_impl ensures it)
        KernelTimer off;
        for (int k = 0; k < 2; ++k) {
            m->cur = k;
            HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            m->step(c->cap_stream, &off);
            HIP_OK(hipStreamEndCapture(c->cap_stream, &m->graph[k]));
            HIP_OK(hipGraphInstantiate(&m->gexec[k], m->graph[k], nullptr, nullptr, 0));
            m->cur = k;
            HIP_OK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < c->opt.graph_steps; ++i) m->step(c->cap_stream, &off);
            HIP_OK(hipStreamEndCapture(c->cap_stream, &m->mgraph[k]));
            HIP_OK(hipGraphInstantiate(&m->mexec[k], m->mgraph[k], nullptr, nullptr, 0));
        }
        m->cur = saved;
        m->keys_fresh = saved_keys;
        m->graph_steps = c->opt.graph_steps;
        m->graphs = true;
    }
    c->step_fn = step_impl<T>;
    c->evaluate_fn = evaluate_impl<T>;
    c->read_fn = read_impl<T>;
    c->nbr_fn = nbr_impl<T>;
    c->closure_fn = closure_impl<T>;
    c->restore_fn = restore_impl<T>;
    c->breakup_fn = breakup_impl<T>;
    c->walls_fn = walls_impl<T>;
    return SPH_OK;
}

}  // namespace

// ------------------------------------------------------------ static workspace
// For callers that cannot allocate device memory: one context per device is
// carved from this array instead of a caller's workspace. Host code never
// passes the array's name to a kernel or a copy; it uses the device address
// that hipGetSymbolAddress returns for the current device (each device holds
// its own copy at its own address).

static __device__ __align__(256) unsigned char scratch[SPH_STATIC_WORKSPACE_BYTES];

namespace {
std::mutex g_static_mu;
std::map<int, void*> g_static_ptr;      // device -> address of its copy of `scratch`
std::map<int, sph_ctx*> g_static_owner; // device -> the live context carved from it
}  // namespace

static void release_static(sph_ctx* c) {
    if (c->static_dev < 0) return;
    std::lock_guard<std::mutex> lk(g_static_mu);
    auto it = g_static_owner.find(c->static_dev);
    if (it != g_static_owner.end() && it->second == c) g_static_owner.erase(it);
    c->static_dev = -1;
}

// ------------------------------------------------------------ C-ABI

extern "C" {

int32_t sph_abi_version(void) { return SPH_ABI_VERSION; }

const char* sph_last_error(const sph_ctx* c) { return c ? c->err.c_str() : g_thread_err.c_str(); }

sph_status sph_workspace_bytes(const sph_options* opt, int32_t n_sys, const sph_params* p,
                               const int64_t* offsets, size_t* bytes_out) {
    sph_ctx* c = nullptr;
    if (!bytes_out) return fail(c, SPH_EINVAL, "bytes_out is NULL");
    sph_options o = resolve(opt);
    std::vector<uint32_t> base;
    if (const char* e = plan(o, n_sys, p, offsets, base)) return fail(c, SPH_EINVAL, e);
    int64_t n = offsets[n_sys];
    bool with_closure = false;
    for (int s = 0; s < n_sys; ++s) with_closure = with_closure || p[s].closure != 0;
    if (o.dtype_bits == 32) {
        Impl<float> m;
        *bytes_out = m.carve(nullptr, n, n_sys, base[n_sys], o.block_stream, with_closure, breakup_bins(n_sys, p),
                             wall_plan(n_sys, p, offsets));
    } else {
        Impl<double> m;
        *bytes_out = m.carve(nullptr, n, n_sys, base[n_sys], o.block_stream, with_closure, breakup_bins(n_sys, p),
                             wall_plan(n_sys, p, offsets));
    }
    return SPH_OK;
}

sph_status sph_init(const sph_options* opt, int32_t n_sys, const sph_params* p, const int64_t* offsets,
                    const double* pos, const double* vel, const double* rho, const double* mass,
                    const int32_t* type, void* d_workspace, size_t ws_bytes, void* stream, sph_ctx** out) {
    sph_ctx* c = nullptr;
    if (!out) return fail(c, SPH_EINVAL, "out is NULL");
    *out = nullptr;
    if (!pos || !vel || !rho || !mass || !type || !d_workspace)
        return fail(c, SPH_EINVAL, "NULL array or workspace");
    sph_options o = resolve(opt);
    std::vector<uint32_t> base;
    if (const char* e = plan(o, n_sys, p, offsets, base)) return fail(c, SPH_EINVAL, e);
    std::unique_ptr<sph_ctx> ctx(new sph_ctx());
    c = ctx.get();
    c->opt = o;
    c->n_sys = n_sys;
    c->n = offsets[n_sys];
    c->stream = static_cast<hipStream_t>(stream);
    c->params.assign(p, p + n_sys);
    c->offsets.assign(offsets, offsets + n_sys + 1);
    c->cell_base = base;
    int rc = o.dtype_bits == 32 ? init_impl<float>(c, pos, vel, rho, mass, type, d_workspace, ws_bytes)
                                : init_impl<double>(c, pos, vel, rho, mass, type, d_workspace, ws_bytes);
    if (rc != SPH_OK) {
        g_thread_err = c->err;
        return (sph_status)rc;
    }
    *out = ctx.release();
    return SPH_OK;
}

sph_status sph_init_static(const sph_options* opt, int32_t n_sys, const sph_params* p, const int64_t* offsets,
                           const double* pos, const double* vel, const double* rho, const double* mass,
                           const int32_t* type, void* stream, sph_ctx** out) {
    sph_ctx* c = nullptr;
    if (!out) return fail(c, SPH_EINVAL, "out is NULL");
    *out = nullptr;
    sph_options o = resolve(opt);
    o.use_graph = 0;   // instantiating a graph may allocate device memory
    size_t need = 0;
    sph_status st = sph_workspace_bytes(&o, n_sys, p, offsets, &need);
    if (st != SPH_OK) return st;
    if (need > (size_t)SPH_STATIC_WORKSPACE_BYTES)
        return fail(c, SPH_ENOMEM, "these systems need " + std::to_string(need) + " bytes of workspace; the static "
                                   "workspace holds " + std::to_string((size_t)SPH_STATIC_WORKSPACE_BYTES));
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (g_static_owner.count(dev))
        return fail(c, SPH_ESTATE, "the static workspace of device " + std::to_string(dev) +
                                   " is held by a live context; sph_free it first");
    void* ptr = nullptr;
    auto it = g_static_ptr.find(dev);
    if (it == g_static_ptr.end()) {
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return fail(c, SPH_EDEVICE, "hipGetSymbolAddress returned a null address");
        g_static_ptr[dev] = ptr;
    } else {
        ptr = it->second;
    }
    st = sph_init(&o, n_sys, p, offsets, pos, vel, rho, mass, type, ptr, (size_t)SPH_STATIC_WORKSPACE_BYTES, stream,
                  out);
    if (st != SPH_OK) return st;
    (*out)->static_dev = dev;
    g_static_owner[dev] = *out;
    return SPH_OK;
}

sph_status sph_step(sph_ctx* c, int32_t n_steps) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    if (n_steps < 0) return fail(c, SPH_EINVAL, "n_steps must be >= 0");
    return (sph_status)c->step_fn(c, n_steps);
}

sph_status sph_evaluate(sph_ctx* c) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    return (sph_status)c->evaluate_fn(c);
}

sph_status sph_read(sph_ctx* c, int32_t field, void* host_dst, size_t bytes) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    return (sph_status)c->read_fn(c, field, host_dst, bytes);
}

sph_status sph_state_bytes(const sph_ctx* c, size_t* bytes_out) {
    if (!c || !bytes_out) return fail(nullptr, SPH_EINVAL, "ctx or bytes_out is NULL");
    *bytes_out = c->opt.dtype_bits == 32 ? state_bytes<float>(c->n, c->n_sys) : state_bytes<double>(c->n, c->n_sys);
    return SPH_OK;
}

sph_status sph_restore(sph_ctx* c, const void* state, size_t bytes) {
    if (!c || !state) return fail(c, SPH_EINVAL, "ctx or state is NULL");
    return (sph_status)c->restore_fn(c, state, bytes);
}

sph_status sph_set_wall_normals(sph_ctx* c, const double* normals) {
    if (!c || !normals) return fail(c, SPH_EINVAL, "ctx or normals is NULL");
    return (sph_status)c->walls_fn(c, normals);
}

sph_status sph_breakup(sph_ctx* c, const double* axis, const double* xi_start, double gap_h, double* length,
                       int32_t* broken) {
    if (!c || !axis || !xi_start || !length || !broken) return fail(c, SPH_EINVAL, "NULL argument");
    if (!isfinite(axis[0]) || !isfinite(axis[1])) return fail(c, SPH_EINVAL, "axis must be finite");
    if (fabs(axis[0] * axis[0] + axis[1] * axis[1] - 1.0) > 1e-12) return fail(c, SPH_EINVAL, "axis must be a unit vector");
    if (!(gap_h >= 1.0) || !isfinite(gap_h)) return fail(c, SPH_EINVAL, "gap_h must be at least 1");
    return (sph_status)c->breakup_fn(c, axis, xi_start, gap_h, length, broken);
}

sph_status sph_neighbors(sph_ctx* c, int64_t* start, int32_t* nbr, int64_t cap, int64_t* total) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    if (!start || !total) return fail(c, SPH_EINVAL, "start/total is NULL");
    return (sph_status)c->nbr_fn(c, start, nbr, cap, total);
}

sph_status sph_sync(sph_ctx* c) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    HIP_OK(hipStreamSynchronize(c->stream));
    return SPH_OK;
}

sph_status sph_profile(sph_ctx* c, int32_t n_steps, int32_t max_stats, const char** names, double* avg_ms,
                       int64_t* calls, int32_t* n_stats) {
    if (!c) return fail(c, SPH_EINVAL, "ctx is NULL");
    if (n_steps < 0 || !n_stats) return fail(c, SPH_EINVAL, "bad arguments");
    c->timer.reset();
    c->timer.enabled = true;
    int rc = SPH_OK;
    if (c->opt.dtype_bits == 32) {
        auto* m = impl_of<float>(c);
        for (int s = 0; s < n_steps; ++s) m->step(c->stream, &c->timer);
    } else {
        auto* m = impl_of<double>(c);
        for (int s = 0; s < n_steps; ++s) m->step(c->stream, &c->timer);
    }
    c->timer.enabled = false;
    c->timer.collect();
    HIP_OK(hipGetLastError());
    c->prof_names = c->timer.names;
    c->prof_ptrs.clear();
    for (auto& s : c->prof_names) c->prof_ptrs.push_back(s.c_str());
    int k = 0;
    for (size_t i = 0; i < c->prof_names.size() && k < max_stats; ++i, ++k) {
        const std::string& nm = c->prof_names[i];
        if (names) names[k] = c->prof_ptrs[i];
        if (avg_ms) avg_ms[k] = c->timer.total_ms[nm] / (double)c->timer.calls[nm];
        if (calls) calls[k] = c->timer.calls[nm];
    }
    *n_stats = (int32_t)c->prof_names.size();
    return (sph_status)rc;
}

sph_status sph_autotune(const sph_options* opt, int32_t n_sys, const sph_params* p, const int64_t* offsets,
                        const double* pos, const double* vel, const double* rho, const double* mass,
                        const int32_t* type, void* d_workspace, size_t ws_bytes, void* stream,
                        int32_t trial_steps, sph_tune_result* out) {
    sph_ctx* c = nullptr;
    if (!out || !p || !offsets || n_sys < 1) return fail(c, SPH_EINVAL, "bad arguments");
    if (trial_steps < 1) return fail(c, SPH_EINVAL, "trial_steps must be >= 1");
    sph_options base = resolve(opt);
    memset(out, 0, sizeof *out);
    // problem class for the cache
    int64_t n = offsets[n_sys];
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= n) ++lg;
    int kernels = 0;
    for (int s = 0; s < n_sys; ++s) kernels |= 1 << p[s].kernel;
    char keybuf[96];
    snprintf(keybuf, sizeof keybuf, "%d/%d/%d/%d", base.dtype_bits, n_sys, lg, kernels);
    static std::map<std::string, sph_tune_result> cache;
    auto hit = cache.find(keybuf);
    if (hit != cache.end()) {
        *out = hit->second;
        out->from_cache = 1;
        out->n_tried = 0;
        return SPH_OK;
    }
    const double factors[] = {1.05, 1.1, 1.2, 2.05, 2.2};
    const int blocks[] = {256, 128};   // the usual winner first: a later one must beat it by 2%
    std::vector<sph_params> q(p, p + n_sys);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(c, SPH_EDEVICE, "hipEventCreate failed");
    double best = 1e300;
    int tried = 0;
    sph_status last = SPH_ENOMEM;
    for (double f : factors) {
        for (int s = 0; s < n_sys; ++s) q[s].cell_size = f * p[s].h;
        for (int bsw : blocks) {
            sph_options o = base;
            o.block_sweep = bsw;
            size_t need = 0;
            if (sph_workspace_bytes(&o, n_sys, q.data(), offsets, &need) != SPH_OK || need > ws_bytes) continue;
            sph_ctx* t = nullptr;
            last = sph_init(&o, n_sys, q.data(), offsets, pos, vel, rho, mass, type, d_workspace, ws_bytes, stream, &t);
            if (last != SPH_OK) continue;
            // two timed windows after a warm-up, the faster one counts
            bool ok = sph_step(t, 2) == SPH_OK;
            double per = 1e300;
            for (int rep = 0; rep < 2 && ok; ++rep) {
                float ms = 0.f;
                ok = hipEventRecord(e0, st) == hipSuccess && sph_step(t, trial_steps) == SPH_OK &&
                     hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                     hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
                if (ok) per = std::min(per, (double)ms / trial_steps);
            }
            sph_free(t);
            if (!ok) continue;
            ++tried;
            // a later candidate must win by more than 2%, so timing noise
            // between near-equal shapes does not flip the choice from run to run
            if (per < (tried == 1 ? 1e300 : 0.98 * best)) {
                best = per;
                out->cell_factor = f;
                out->block_sweep = bsw;
                out->ms_per_step = per;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!tried) return fail(c, last == SPH_OK ? SPH_ENOMEM : last, "no configuration could be timed");
    out->n_tried = tried;
    cache[keybuf] = *out;
    return SPH_OK;
}

sph_status sph_set_closure(sph_ctx* c, const float* params) {
    if (!c || !params) return fail(c, SPH_EINVAL, "ctx or params is NULL");
    return (sph_status)c->closure_fn(c, params);
}

// ------------------------------------------------------------ closure trainer

static size_t mlp_carve(sph_mlp* t, char* base, int64_t max_batch) {
    Carver cv{base};
    const int nw = mlp_grad_waves(max_batch);
    MlpBufs B{};
    B.master = cv.take<float>(MLP_NPARAMS);
    B.adam_m = cv.take<float>(MLP_NPARAMS);
    B.adam_v = cv.take<float>(MLP_NPARAMS);
    B.wt1 = cv.take<uint16_t>(64 * 64);
    B.wt2 = cv.take<uint16_t>(64 * 64);
    B.wt3 = cv.take<uint16_t>(16 * 64);
    B.w2 = cv.take<uint16_t>(64 * 64);
    B.w3 = cv.take<uint16_t>(64 * 16);
    B.b1 = cv.take<float>(64);
    B.b2 = cv.take<float>(64);
    B.b3 = cv.take<float>(16);
    float* grad = cv.take<float>(MLP_NPARAMS);
    float* loss = cv.take<float>(4);
    float* partial = cv.take<float>((size_t)nw * MLP_NPARAMS);
    float* loss_part = cv.take<float>(nw);
    float* staging = cv.take<float>(MLP_NPARAMS);
    if (t) {
        t->B = B;
        t->grad = grad;
        t->loss = loss;
        t->partial = partial;
        t->loss_part = loss_part;
        t->staging = staging;
    }
    return cv.off + 256;
}

sph_status sph_mlp_workspace_bytes(int64_t max_batch, size_t* bytes_out) {
    sph_ctx* c = nullptr;
    if (!bytes_out || max_batch < 1) return fail(c, SPH_EINVAL, "bad arguments");
    *bytes_out = mlp_carve(nullptr, nullptr, max_batch);
    return SPH_OK;
}

sph_status sph_mlp_create(const float* params, int64_t max_batch, void* d_workspace, size_t ws_bytes, void* stream,
                          sph_mlp** out) {
    sph_ctx* c = nullptr;
    if (!out || !params || !d_workspace || max_batch < 1) return fail(c, SPH_EINVAL, "bad arguments");
    *out = nullptr;
    if (mlp_carve(nullptr, nullptr, max_batch) > ws_bytes) return fail(c, SPH_ENOMEM, "workspace too small");
    if (((uintptr_t)d_workspace) & 255) return fail(c, SPH_EINVAL, "workspace must be 256-byte aligned");
    std::unique_ptr<sph_mlp> t(new sph_mlp());
    t->stream = static_cast<hipStream_t>(stream);
    t->max_batch = max_batch;
    mlp_carve(t.get(), static_cast<char*>(d_workspace), max_batch);
    hipStream_t st = t->stream;
    launch_fill_u32(reinterpret_cast<uint32_t*>(t->B.adam_m), MLP_NPARAMS, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(t->B.adam_v), MLP_NPARAMS, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(t->B.wt3), 16 * 64 / 2, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(t->B.w3), 64 * 16 / 2, 0u, st);
    launch_fill_u32(reinterpret_cast<uint32_t*>(t->B.b3), 16, 0u, st);
    HIP_OK(hipMemcpyAsync(t->staging, params, sizeof(float) * MLP_NPARAMS, hipMemcpyHostToDevice, st));
    launch_mlp_set(t->B, t->staging, st);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(st));
    *out = t.release();
    return SPH_OK;
}

sph_status sph_mlp_forward(sph_mlp* t, const uint16_t* d_x, int64_t m, float* d_y) {
    sph_ctx* c = nullptr;
    if (!t || !d_x || !d_y || m < 0) return fail(c, SPH_EINVAL, "bad arguments");
    if (m > 0) launch_mlp_forward(t->B.view(), d_x, m, d_y, 3, t->stream);
    HIP_OK(hipGetLastError());
    return SPH_OK;
}

sph_status sph_mlp_gradient(sph_mlp* t, const uint16_t* d_x, const float* d_t, int64_t m, float* d_grad,
                            float* d_loss) {
    sph_ctx* c = nullptr;
    if (!t || !d_x || !d_t || !d_grad || m < 1 || m > t->max_batch) return fail(c, SPH_EINVAL, "bad arguments");
    launch_mlp_grad(t->B.view(), d_x, d_t, m, t->partial, t->loss_part, d_grad, d_loss,
                    t->stream);
    HIP_OK(hipGetLastError());
    return SPH_OK;
}

sph_status sph_mlp_train_step(sph_mlp* t, const uint16_t* d_x, const float* d_t, int64_t m, float lr,
                              float* d_loss) {
    sph_ctx* c = nullptr;
    if (!t || !d_x || !d_t || m < 1 || m > t->max_batch || !(lr > 0)) return fail(c, SPH_EINVAL, "bad arguments");
    launch_mlp_grad(t->B.view(), d_x, d_t, m, t->partial, t->loss_part, t->grad,
                    d_loss ? d_loss : t->loss, t->stream);
    t->t += 1;
    launch_mlp_adam(t->B, t->grad, lr, t->t, t->stream);
    HIP_OK(hipGetLastError());
    return SPH_OK;
}

sph_status sph_mlp_params(sph_mlp* t, float* params) {
    sph_ctx* c = nullptr;
    if (!t || !params) return fail(c, SPH_EINVAL, "bad arguments");
    HIP_OK(hipMemcpyAsync(params, t->B.master, sizeof(float) * MLP_NPARAMS, hipMemcpyDeviceToHost, t->stream));
    HIP_OK(hipStreamSynchronize(t->stream));
    return SPH_OK;
}

void sph_mlp_free(sph_mlp* t) {
    if (!t) return;
    (void)hipStreamSynchronize(t->stream);
    delete t;
}

void sph_free(sph_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    c->impl.reset();
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    release_static(c);
    delete c;
}

}  // extern "C"

// Internal declarations shared by the kernels and the host side of libsphjet.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <vector>

#include "sph_device.hpp"

namespace sphjet {

// Position arrays hold this many slots past the last particle: the candidate
// scan loads four positions from one address and may run over a row's end.
constexpr int POS_PAD = 4;

// The surface list of an evaluation is split into this many regions, each
// with its own counter, so its appends do not all contend for one address.
constexpr int SURF_REGIONS = 64;
constexpr int SURF_BLOCK = 32;   // consecutive sweep chunks that share a region
// Surface lists of at most this many entries (fewer than one 64-lane wave per
// SIMD of the chip at one lane per entry) give each entry four lanes in the
// surface sweep.
constexpr uint32_t SURF_SPLIT_MAX = 65536;

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// One full set of per-slot state arrays.
template <typename T>
struct StateBuf {
    double2* pos;
    V2<T>* vel;
    T* dens;
    T* mass;
    uint32_t* tag;
    uint32_t* id;
};

struct SortBufs {
    uint32_t trash;     // number of cells of all systems = key of inactive particles
    uint32_t* count;    // trash + 1: particles per cell (key kernel); zero between sorts
    uint32_t* cstart;   // trash + 2: first slot of every cell (+ inactive start + end)
    uint32_t* key;      // n: key of each slot before the sort
    uint32_t* slot;     // n: position inside its cell (atomic order)
    uint32_t* blk;      // workgroups + 1: inactive counts, then their offsets
    uint32_t* part;     // tile sums of the cell scan
    uint32_t* part2;    // tile sums of the workgroup scan
    uint32_t* cell_ids; // n: ids of every cell's particles in its slot range (unordered)
    uint32_t* scratch;  // n: free between steps (neighbour counts of sph_neighbors)
    uint32_t* cell;     // n: cell key of each sorted slot
    uint32_t* sys_cell_base;  // n_sys + 1: first cell of every system (last = trash)
    uint32_t* sys_lo;         // n_sys: first sorted slot of every system
    uint32_t* sys_hi;         // n_sys: one past its last active slot
    uint32_t* chunk_base;     // n_sys + 1: first 64-slot wave chunk of every system
    uint32_t* surf_count;     // SURF_REGIONS surface-list counters (cleared with the wave table)
};

// Repulsive-force walls of one system: two static cell grids (fixed walls,
// then pistons) of the boundary particles' positions (pistons at their travel
// x_ref) and normals, built on the host by sph_set_wall_normals.
struct WallSys {
    double x0, y0, inv_cs, db, x_ref;
    int32_t nx, ny;
    uint32_t cell_base[2];   // first cell-start entry of each grid
};

struct WallView {
    const WallSys* sys;
    const uint32_t* cstart;  // per cell of every grid: first record (+ one past the last)
    const double4* rec;      // x, y, n_x, n_y
    const double* time;      // the systems' time and last dt: the evaluation's time
    const double* dt;
    int half;                // 1 in the half-step evaluation
    int pad_;
};

// What the three sweeps read and write.
template <typename T>
struct EvalView {
    int n;
    int xcd;
    int do_dt;
    int n_sys;
    const uint32_t* sys_lo;
    const uint32_t* sys_hi;
    const uint32_t* chunk_base;
    const SysDev<T>* sys;
    const double2* pos;
    const V2<T>* vel;
    const T* dens;
    const T* mass;
    const uint32_t* tag;
    const uint32_t* id;
    const uint32_t* cell;
    const uint32_t* cstart;
    T* colour;
    T* drho;
    V2<T>* acc;
    V2<T>* nrm;
    T* kappa;
    T* kappa_plain;
    unsigned long long* dtmin;  // 2 per system: [h/(c+sig) min, sqrt(h/|a|) min] (atomic minima)
    double* dt_wave;            // 2 per sweep chunk: the main sweep's wave minima of the same
    const T* vol;               // m / rho of every slot (this evaluation's state)
    V4<T>* eos;                 // (P / rho^2, colour, rho, m / rho), written by the colour sweep
    uint4* nmask;                // n: neighbour mask words of cell rows 0..3 (the mask the sweeps walk)
    uint32_t* nmask4;            // n: word of row 4 (+ overflow bit 31)
    uint4* smask;                // n: where the first colour sweep writes the skin mask (pairs within
    uint32_t* smask4;            //   R s); null in the half-step evaluation
    int pad3_;
    // half-step evaluation only (else null): per system, then over all
    // systems, the bit pattern of the largest squared half-step displacement
    // beyond half the skin (0: none); such a system's sweeps scan the
    // step-start cells with a wider reach
    const unsigned long long* skin_max;
    uint32_t* flags;
    T* dens_out;                 // the evaluation's density (= dens), written by the density summation
    T* vol_out;                  // its m / rho (= vol)
    int density_sum;             // some system uses the density summation (eq. 6)
    int pad4_;
    V2<T>* fwall;                // repulsive-force walls: force per unit mass on each fluid slot
    uint32_t* cl_count;          // closure list (null when no system uses the closure)
    uint32_t* cl_list;
    uint32_t cl_capacity;
    uint32_t surf_region;        // capacity of one region of the surface list
    uint32_t* surf_count;        // SURF_REGIONS counters (cleared by the wave table and the predictor)
    uint32_t* surf_list;         // SURF_REGIONS regions: slots that pass the normal filter
};

// Learned closure network: parameter count and offsets of the flat FP32
// parameter vector (W1 in x out row-major, b1, W2, b2, W3 64 x 3, b3).
constexpr int MLP_OFF_W1 = 0;
constexpr int MLP_OFF_B1 = 64 * 64;
constexpr int MLP_OFF_W2 = MLP_OFF_B1 + 64;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + 64 * 64;
constexpr int MLP_OFF_W3 = MLP_OFF_B2 + 64;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + 64 * 3;
constexpr int MLP_NPARAMS = MLP_OFF_B3 + 3;

// BF16 working copies read by the network kernels: wt* transposed (out x in),
// w2 and w3 as stored (in x out, w3 padded to 16 outputs); FP32 biases (b3
// padded to 16).
struct MlpView {
    const uint16_t* wt1;
    const uint16_t* wt2;
    const uint16_t* wt3;
    const uint16_t* w2;
    const uint16_t* w3;
    const float* b1;
    const float* b2;
    const float* b3;
};

// Everything the trainer owns on the device.
struct MlpBufs {
    float* master;   // MLP_NPARAMS FP32 masters
    float* adam_m;
    float* adam_v;
    uint16_t* wt1;   // 64 x 64
    uint16_t* wt2;   // 64 x 64
    uint16_t* wt3;   // 16 x 64 (rows 3..15 zero)
    uint16_t* w2;    // 64 x 64
    uint16_t* w3;    // 64 x 16 (columns 3..15 zero)
    float* b1;       // 64
    float* b2;       // 64
    float* b3;       // 16 (3..15 zero)
    MlpView view() const { return MlpView{wt1, wt2, wt3, w2, w3, b1, b2, b3}; }
};

// The closure's per-evaluation buffers.
struct ClosureView {
    uint32_t* count;     // surface particles listed this evaluation
    uint32_t* list;      // their slots
    uint16_t* stencil;   // 64 BF16 per listed particle
    float* out;          // 4 per listed particle: n_x, n_y, kappa h, unused
    uint32_t* fallback;  // per slot: 1 where the plain curvature was used
    uint32_t capacity;
    uint32_t quad_min;   // listed counts above this build four stencils per wave
};

// What the predictor and corrector read and write.
template <typename T>
struct IntegView {
    int n;
    int n_sys;
    const SysDev<T>* sys;
    double2* pos;          // state n (corrector updates it in place)
    V2<T>* vel;
    T* dens;
    uint32_t* tag;
    const T* mass;
    const T* drho;         // derivatives of the last evaluation
    const V2<T>* acc;
    double2* pos_h;        // half-step state (predictor output)
    V2<T>* vel_h;
    T* dens_h;
    const double* dt;
    const double* time;
    uint32_t* flags;
    T* vol;                // m / rho of the half-step state
    uint32_t* surf_count;  // surface-list counters, cleared for the half-step evaluation
    unsigned long long* skin_max;  // per system, then over all: largest squared half-step displacement
                                   // beyond half the skin (0: none)
    // corrector only: the next sort's keys, slots, cell counts and workgroup
    // inactive counts of the new state (key == nullptr: not written)
    uint32_t* key;
    uint32_t* kslot;
    uint32_t* kcount;
    uint32_t* kblk;
    uint32_t trash;
};

struct LaunchCfg {
    int n;
    int n_sys;
    int block_sweep;
    int block_stream;
    int xcd;
};

// Optional per-kernel timing with HIP events on the launch stream.
class KernelTimer {
public:
    bool enabled = false;
    void begin(const char* name, hipStream_t st);
    void end(hipStream_t st);
    // Waits for the events and accumulates elapsed times per name.
    void collect();
    void reset();
    std::vector<std::string> names;
    std::map<std::string, double> total_ms;
    std::map<std::string, long long> calls;
    ~KernelTimer();

private:
    struct Pending { std::string name; hipEvent_t a, b; };
    std::vector<Pending> pending_;
    std::vector<hipEvent_t> pool_;
    hipEvent_t get_();
    const char* cur_ = nullptr;
    hipEvent_t cur_a_ = nullptr;
};

void launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st);
int64_t scan_tiles(int64_t m);
int64_t surface_region(int64_t n, int n_sys);   // slots of one surface-list region
int64_t surface_chunks(int64_t n, int n_sys);   // bound on the sweeps' 64-slot chunks
void launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t st);
void copy_kernel(const void* src, void* dst, size_t bytes, hipStream_t st);

template <typename T>
void launch_key(const LaunchCfg& L, const SortBufs& B, const SysDev<T>* sys, StateBuf<T> X, hipStream_t st,
                KernelTimer* kt);
// keyed: X's keys, slots and cell counts are already written (by the corrector)
template <typename T>
void launch_sort(const LaunchCfg& L, const SortBufs& B, const SysDev<T>* sys, StateBuf<T> X, StateBuf<T> Y,
                 T* vol, bool keyed, hipStream_t st, KernelTimer* kt);
template <typename T>
void launch_eval(const LaunchCfg& L, const EvalView<T>& v, const WallView* W, hipStream_t st, KernelTimer* kt);
template <typename T>
void launch_dt(int n_sys, const SysDev<T>* sys, const uint32_t* chunk_base, const double* dt_wave,
               unsigned long long* dtmin, double* dt, unsigned long long* skin_max, hipStream_t st,
               KernelTimer* kt);
template <typename T>
void launch_predict(const LaunchCfg& L, const IntegView<T>& v, hipStream_t st, KernelTimer* kt);
template <typename T>
void launch_correct(const LaunchCfg& L, const IntegView<T>& v, int n_sys, const double* dt, double* time,
                    hipStream_t st, KernelTimer* kt);
template <typename T>
void launch_colour_mask(const LaunchCfg& L, const EvalView<T>& v, hipStream_t st);
template <typename T>
void launch_nbr_count(const LaunchCfg& L, const EvalView<T>& v, uint32_t* count, hipStream_t st);
template <typename T>
void launch_nbr_fill(const EvalView<T>& v, int a0, int a1, const int64_t* start, int64_t base, uint32_t* out,
                     hipStream_t st);
template <typename T>
void launch_pressure(int n, const SysDev<T>* sys, const uint32_t* tag, const T* dens, T* out, hipStream_t st);
// Breakup length: per-system extent along the axis, then the binned gap search.
void launch_breakup(int n, int n_sys, const uint32_t* tag, const double2* pos, double ax, double ay,
                    const double* start, unsigned long long* extent, hipStream_t st);
void launch_breakup_bins(int n, int n_sys, const uint32_t* tag, const double2* pos, double ax, double ay,
                         const double* start, const double* anchor, const double* half_gap, const double* gap,
                         const uint32_t* bin_base, uint32_t n_bins, unsigned long long* bmin, unsigned long long* bmax,
                         double* length, int32_t* broken, hipStream_t st);

void launch_mlp_forward(const MlpView& W, const uint16_t* X, int64_t m, float* Y, int ystride, hipStream_t st);
constexpr int MLP_GRAD_WAVES = 1024;
int mlp_grad_waves(int64_t m);
void launch_mlp_grad(const MlpView& W, const uint16_t* X, const float* T, int64_t m, float* partial,
                     float* loss_part, float* grad, float* loss, hipStream_t st);
void launch_mlp_set(const MlpBufs& B, const float* params, hipStream_t st);
void launch_mlp_adam(const MlpBufs& B, const float* grad, float lr, int t, hipStream_t st);
template <typename T>
void launch_closure(const EvalView<T>& v, const ClosureView& C, const MlpView& W, int64_t capacity, hipStream_t st,
                    KernelTimer* kt);

}  // namespace sphjet

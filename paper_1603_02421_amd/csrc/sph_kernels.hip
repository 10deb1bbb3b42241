// HIP kernels of libsphjet (gfx950). One thread per particle slot throughout;
// every per-particle sum is a gather over the slot ranges of the neighbouring
// cells, so no floating-point atomics are used and results are bit-for-bit
// reproducible run to run.
#include <type_traits>

#include "sph_internal.hpp"

namespace sphjet {

// ------------------------------------------------------------------ helpers

__global__ void k_fill_u32(uint32_t* p, size_t n, uint32_t v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, size_t n, unsigned long long v) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan inside one workgroup of SCAN_THREADS threads (wave64 shuffles
// + one LDS pass over the wave totals). Returns the exclusive prefix of x and
// writes the workgroup total to *total.
__device__ uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
    __shared__ uint32_t wsum[17];
    const int lane = __lane_id(), wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int w = 0; w < nw; ++w) { uint32_t t = wsum[w]; wsum[w] = run; run += t; }
        wsum[16] = run;
    }
    __syncthreads();
    uint32_t r = wsum[wid] + incl - x;
    *total = wsum[16];
    __syncthreads();
    return r;
}

// ------------------------------------------------------------------ scan (u32)
// Exclusive prefix sum out[i] = sum of in[0..i), out[m] = the total. Large
// arrays take three passes over tiles of SCAN_TILE elements (tile sums, one
// workgroup scanning the tile sums, apply); small ones one workgroup. Every
// thread owns SCAN_ITEMS consecutive elements, loaded and stored as uint4.
// With clear_in the apply pass zeroes the input after reading it, so the cell
// counts are ready for the next sort without a separate clear.

// The SCAN_ITEMS elements of this thread starting at i0 (zeros past m).
__device__ __forceinline__ void scan_load(const uint32_t* in, int64_t i0, int64_t m, uint32_t* v) {
    if (i0 + SCAN_ITEMS <= m) {
#pragma unroll
        for (int u = 0; u < SCAN_ITEMS / 4; ++u) {
            const uint4 q = reinterpret_cast<const uint4*>(in + i0)[u];
            v[4 * u] = q.x;
            v[4 * u + 1] = q.y;
            v[4 * u + 2] = q.z;
            v[4 * u + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) v[k] = i0 + k < m ? in[i0 + k] : 0u;
    }
}

// out[i0 + k] = run + v[0] + ... + v[k - 1] (elements below m); returns the
// running sum past the last element.
__device__ __forceinline__ uint32_t scan_store(uint32_t* out, int64_t i0, int64_t m, const uint32_t* v, uint32_t run) {
    if (i0 + SCAN_ITEMS <= m) {
#pragma unroll
        for (int u = 0; u < SCAN_ITEMS / 4; ++u) {
            uint4 o;
            o.x = run;
            run += v[4 * u];
            o.y = run;
            run += v[4 * u + 1];
            o.z = run;
            run += v[4 * u + 2];
            o.w = run;
            run += v[4 * u + 3];
            reinterpret_cast<uint4*>(out + i0)[u] = o;
        }
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            if (i0 + k < m) out[i0 + k] = run;
            run += v[k];
        }
    }
    return run;
}

// Zero the elements of this thread that were non-zero.
__device__ __forceinline__ void scan_clear(uint32_t* in, int64_t i0, int64_t m, const uint32_t* v) {
    if (i0 + SCAN_ITEMS <= m) {
#pragma unroll
        for (int u = 0; u < SCAN_ITEMS / 4; ++u)
            if (v[4 * u] | v[4 * u + 1] | v[4 * u + 2] | v[4 * u + 3])
                reinterpret_cast<uint4*>(in + i0)[u] = make_uint4(0u, 0u, 0u, 0u);
    } else {
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k)
            if (i0 + k < m && v[k]) in[i0 + k] = 0u;
    }
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_reduce(const uint32_t* in, int64_t m, uint32_t* part) {
    const int64_t i0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    scan_load(in, i0, m, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// One workgroup (up to 1024 threads) scans all of in[0..m) in chunks of
// blockDim.x * SCAN_ITEMS, carrying the running total from chunk to chunk.
__global__ void __launch_bounds__(1024) k_scan_single(uint32_t* in, uint32_t* out, int64_t m) {
    const int64_t tile = (int64_t)blockDim.x * SCAN_ITEMS;
    uint32_t carry = 0;
    for (int64_t base = 0; base < m; base += tile) {
        const int64_t i0 = base + (int64_t)threadIdx.x * SCAN_ITEMS;
        uint32_t v[SCAN_ITEMS];
        scan_load(in, i0, m, v);
        uint32_t s = 0;
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
        uint32_t tot;
        const uint32_t excl = block_exclusive_scan(s, &tot);
        scan_store(out, i0, m, v, carry + excl);
        carry += tot;
    }
    if (threadIdx.x == 0) out[m] = carry;
}

__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(uint32_t* in, uint32_t* out, int64_t m,
                                                           const uint32_t* part, int clear_in) {
    const int64_t i0 = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    scan_load(in, i0, m, v);
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) s += v[k];
    if (clear_in && s) scan_clear(in, i0, m, v);
    uint32_t tot;
    const uint32_t excl = block_exclusive_scan(s, &tot);
    const uint32_t run = scan_store(out, i0, m, v, part[blockIdx.x] + excl);
    if (i0 < m && i0 + SCAN_ITEMS >= m) out[m] = run;   // the thread holding element m - 1
}

// ------------------------------------------------------------------ sort
// Cell key of every slot, slot within its cell (atomic counter: only a place
// for the particle's id, the order inside a cell is fixed by k_permute), and
// per-workgroup counts of particles outside the cells -- inactive ones and the
// walls of repulsive-force systems -- whose order comes from a stable
// compaction.

// Every thread of the workgroup calls it (valid = slot i < n), with the
// particle's tag and position: the key goes to key[i], the slot within the
// cell to slot[i], and the workgroup's count of particles outside the cells
// to blk_inactive[blockIdx.x].
template <typename T>
__device__ __forceinline__ void key_and_count(const SysDev<T>* sys, int i, bool valid, uint32_t t, double2 p,
                                              uint32_t* key, uint32_t* slot, uint32_t* counts, uint32_t trash,
                                              uint32_t* blk_inactive) {
    bool inactive = false, act = false;
    uint32_t k = trash;
    if (valid) {
        // repulsive-force walls stay out of the cells, like inactive particles:
        // they act on the fluid only through the wall force (eq. 29)
        if (tag_type(t) != T_INACTIVE && !(sys[tag_sys(t)].boundary && tag_type(t) != T_FLUID)) {
            const SysDev<T>& S = sys[tag_sys(t)];
            int cx = cell_coord(p.x, S.x0, S.inv_s, S.nx);
            int cy = cell_coord(p.y, S.y0, S.inv_s, S.ny);
            k = S.cell_base + (uint32_t)cx * (uint32_t)S.ny + (uint32_t)cy;
            act = true;
        } else {
            inactive = true;
        }
    }
    // One atomic per run of consecutive lanes with the same key: the head of
    // the run reserves the run's slots, members take consecutive ones.
    const int lane = __lane_id();
    const uint32_t kk = act ? k : 0xFFFFFFFFu;
    const uint32_t prev = __shfl_up(kk, 1, 64);
    const bool head = act && (lane == 0 || prev != kk);
    const unsigned long long heads = __ballot(head);
    const unsigned long long actm = __ballot(act);
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const unsigned long long hm = heads & upto;
    const int hlane = hm ? 63 - __clzll((long long)hm) : lane;
    uint32_t base = 0;
    if (head) {
        const unsigned long long brk = (heads | ~actm) & (lane == 63 ? 0ull : (~0ull << (lane + 1)));
        const int next = brk ? __ffsll((long long)brk) - 1 : 64;
        base = atomicAdd(&counts[k], (uint32_t)(next - lane));
    }
    base = __shfl(base, hlane, 64);
    if (valid) {
        key[i] = k;
        slot[i] = act ? base + (uint32_t)(lane - hlane) : 0u;
    }
    int c = __syncthreads_count(inactive);
    if (threadIdx.x == 0) blk_inactive[blockIdx.x] = (uint32_t)c;
}

template <typename T>
__global__ void k_key(int n, const SysDev<T>* sys, const double2* pos, const uint32_t* tag,
                      uint32_t* key, uint32_t* slot, uint32_t* counts, uint32_t trash,
                      uint32_t* blk_inactive) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < n;
    const uint32_t t = valid ? tag[i] : 0u;
    const double2 p = valid ? pos[i] : make_double2(0.0, 0.0);
    key_and_count<T>(sys, i, valid, t, p, key, slot, counts, trash, blk_inactive);
}

// The ids of every cell's particles, in the cell's slot range (in the
// arbitrary order of the key kernel's atomics).
__global__ void k_scatter(int n, const uint32_t* key, const uint32_t* slot, const uint32_t* id,
                          const uint32_t* cstart, uint32_t trash, uint32_t* cell_ids) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t k = key[i];
    if (k != trash) cell_ids[cstart[k] + slot[i]] = id[i];
}

// Move every particle to its slot of the sorted order, which is (cell key,
// particle id): the first slot of its cell plus the number of the cell's
// particles with a smaller id (ids are unique). Inactive particles follow all
// cells in their previous order (stable compaction per workgroup, the same
// workgroups as the key kernel). Also m / rho for the first evaluation of the
// step.
template <typename T>
__global__ void k_permute(int n, const SysDev<T>* sys, const uint32_t* key, const uint32_t* cstart,
                          const uint32_t* cell_ids, uint32_t trash, const uint32_t* blk_off, StateBuf<T> X,
                          StateBuf<T> Y, uint32_t* cell, T* vol) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k = i < n ? key[i] : 0u;
    const bool inactive = i < n && k == trash;
    // the particle's state is loaded before the compaction scan and the rank
    // search, so those loads overlap their latency
    const int j = i < n ? i : 0;
    const double2 p = X.pos[j];
    const V2<T> u = X.vel[j];
    const T dens = X.dens[j], mass = X.mass[j];
    const uint32_t t = X.tag[j], pid = X.id[j];
    uint32_t tot;
    const uint32_t rank = block_exclusive_scan(inactive ? 1u : 0u, &tot);
    if (i >= n) return;
    uint32_t dst;
    if (inactive) {
        dst = cstart[trash] + blk_off[blockIdx.x] + rank;
    } else {
        const uint32_t lo = cstart[k], hi = cstart[k + 1];
        uint32_t r = 0;
        for (uint32_t j = lo; j < hi; ++j) r += cell_ids[j] < pid ? 1u : 0u;
        dst = lo + r;
    }
    Y.pos[dst] = p;
    Y.vel[dst] = u;
    Y.dens[dst] = dens;
    Y.mass[dst] = mass;
    Y.tag[dst] = t;
    Y.id[dst] = pid;
    cell[dst] = k;
    if (!inactive) vol[dst] = particle_vol(sys[tag_sys(t)], dens, mass);
}

// ------------------------------------------------------------------ sweeps
// Work assignment: every wavefront owns up to 64 consecutive slots of a single
// system (the wave table is rebuilt after every sort), so the system's
// constants are wave-uniform and live in scalar registers.

__global__ void __launch_bounds__(1024) k_wave_table(int n_sys, const uint32_t* cell_base, const uint32_t* cstart,
                                                    uint32_t* sys_lo, uint32_t* sys_hi, uint32_t* chunk_base,
                                                    uint32_t* surf_count) {
    if (threadIdx.x < SURF_REGIONS) surf_count[threadIdx.x] = 0u;   // the first evaluation's surface list
    int per = (n_sys + 1023) / 1024;
    int s0 = (int)threadIdx.x * per, s1 = s0 + per < n_sys ? s0 + per : n_sys;
    uint32_t sum = 0;
    for (int s = s0; s < s1; ++s) {
        uint32_t lo = cstart[cell_base[s]], hi = cstart[cell_base[s + 1]];
        sys_lo[s] = lo;
        sys_hi[s] = hi;
        sum += (hi - lo + 63u) >> 6;
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(sum, &tot);
    for (int s = s0; s < s1; ++s) {
        chunk_base[s] = run;
        run += (sys_hi[s] - sys_lo[s] + 63u) >> 6;
    }
    if (threadIdx.x == 0) chunk_base[n_sys] = tot;
}

// The system and slot of this lane; false (for the whole wave) when the wave
// has no chunk. Slots past the end of the system are not valid.
template <typename T>
__device__ __forceinline__ bool wave_assign(const EvalView<T>& v, int& sys, uint32_t& a, uint32_t* chunk = nullptr) {
    const int wpb = (int)(blockDim.x >> 6);
    const uint32_t wave = (uint32_t)(tile_index(v.xcd) * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6));
    if (chunk) *chunk = wave;
    const uint32_t total = v.chunk_base[v.n_sys];
    if (wave >= total) return false;
    int lo = 0, hi = v.n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (v.chunk_base[mid] <= wave) lo = mid;
        else hi = mid - 1;
    }
    sys = __builtin_amdgcn_readfirstlane(lo);
    a = v.sys_lo[sys] + (wave - v.chunk_base[sys]) * 64u + (uint32_t)__lane_id();
    return true;
}

// Minimum of non-negative values over the wave into dst (one system per wave).
__device__ __forceinline__ void wave_atomic_min(unsigned long long* dst, double v, bool valid) {
    double m = wave_min(valid ? v : __builtin_inf());
    if (__lane_id() == 0 && m < __builtin_inf()) atomic_min_bits(dst, m);
}

// Visit every slot b != a of the (2R+1)^2 cells around slot a's cell that
// passes the exact predicate |r_ab|^2 < rp2 (rp2 = (2h)^2 for the neighbours,
// (R s)^2 for the skin mask of the colour sweep). R is the system's reach,
// or a wider one when the half step rescans (rescan_reach). Candidates are taken four at a
// time: their positions are loaded together, then the per-neighbour payload of
// the accepted ones (load(b)), then compute(b, k, dx, dy, r2, payload) with k
// the slot's place in its cell row, r_ab = r_a - r_b in the working precision
// and r2 = |r_ab|^2 as the predicate formed it (FP64). Slot ranges come
// straight from the cell starts: with the y index fastest, each cell row is
// one range.
template <typename T, int NB = 4, typename LoadFn, typename ComputeFn, typename RowEndFn>
__device__ __forceinline__ void scan_cells_rows(const SysDev<T>& S, const uint32_t* __restrict__ cstart, uint32_t cell,
                                                uint32_t a, double2 pa, const double2* __restrict__ pos, LoadFn&& load,
                                                ComputeFn&& compute, RowEndFn&& row_end, double rp2, int R) {
    using P = typename std::decay<decltype(load(0u))>::type;
    const uint32_t ny = (uint32_t)S.ny;
    const uint32_t local = cell - S.cell_base;
    const int cx = (int)(local / ny);
    const int cy = (int)(local - (uint32_t)cx * ny);
    const int ylo = cy - R < 0 ? 0 : cy - R;
    const int yhi = cy + R > S.ny - 1 ? S.ny - 1 : cy + R;
    const int xlo = cx - R < 0 ? 0 : cx - R;
    const int xhi = cx + R > S.nx - 1 ? S.nx - 1 : cx + R;
    const double R2 = rp2;
    // the rows' slot ranges, loaded together before the scan (reach <= 2
    // here, so at most five rows; wider rescans load each row's in turn)
    uint32_t rb0[5], rb1[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        const int X = xlo + i;
        const bool in = X <= xhi && R <= 2;
        const uint32_t row = S.cell_base + (uint32_t)(in ? X : xlo) * ny;
        rb0[i] = in ? cstart[row + ylo] : 0u;
        rb1[i] = in ? cstart[row + yhi + 1] : 0u;
    }
    int r = 0;   // row of the block, 0 at x = xlo
    for (int X = xlo; X <= xhi; ++X, ++r) {
        const uint32_t row = S.cell_base + (uint32_t)X * ny;
        uint32_t b0, b1;
        if (R <= 2) {
            b0 = r == 0 ? rb0[0] : r == 1 ? rb0[1] : r == 2 ? rb0[2] : r == 3 ? rb0[3] : rb0[4];
            b1 = r == 0 ? rb1[0] : r == 1 ? rb1[1] : r == 2 ? rb1[2] : r == 3 ? rb1[3] : rb1[4];
        } else {
            b0 = cstart[row + ylo];
            b1 = cstart[row + yhi + 1];
        }
        for (uint32_t b = b0; b < b1; b += NB) {
            // NB positions from one address: the position arrays hold
            // POS_PAD slots past the last particle, so a batch may run over
            // the end of the row (those candidates fail the b + k < b1 test)
            const double2* pb = pos + b;
            double2 q[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) q[k] = pb[k];
            bool ok[NB];
            T dx[NB], dy[NB];
            double r2[NB];
#pragma unroll
            for (int k = 0; k < NB; ++k) {
                double ex, ey;
                r2[k] = pair_r2(pa, q[k], ex, ey);
                ok[k] = (b + k < b1) && (b + k != a) && (r2[k] < R2);
                dx[k] = (T)ex;
                dy[k] = (T)ey;
            }
            P pl[NB] = {};
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (ok[k]) pl[k] = load(b + k);
#pragma unroll
            for (int k = 0; k < NB; ++k)
                if (ok[k]) compute(b + k, b + k - b0, dx[k], dy[k], r2[k], pl[k]);
        }
        row_end(r);
    }
}

template <typename T, int NB = 4, typename LoadFn, typename ComputeFn>
__device__ __forceinline__ void scan_cells(const SysDev<T>& S, const uint32_t* __restrict__ cstart, uint32_t cell,
                                           uint32_t a, double2 pa, const double2* __restrict__ pos, LoadFn&& load,
                                           ComputeFn&& compute, int R) {
    scan_cells_rows<T, NB>(S, cstart, cell, a, pa, pos, load,
                           [&](uint32_t b, uint32_t, T dx, T dy, double, const auto& p) { compute(b, dx, dy, p); },
                           [](int) {}, S.R2, R);
}

// Reach of a half-step rescan of system `sys`, 0 when its particles all stayed
// within half the skin (the skin mask is complete). A pair within 2h at the
// half step was within 2h + 2d at the step start, d the system's largest
// half-step displacement, so its cells differ by at most ceil((2h + 2d)/s) in
// each direction. Beyond RESCAN_MAX_REACH the scan keeps that reach and
// FLAG_SKIN reports that pairs may be missing.
template <typename T>
__device__ __forceinline__ int rescan_reach(const EvalView<T>& v, const SysDev<T>& S, int sys) {
    if (!v.skin_max) return 0;
    const unsigned long long bits = v.skin_max[sys];
    if (!bits) return 0;
    const double d = sqrt(__longlong_as_double((long long)bits));
    const double need = ceil((sqrt(S.R2) + 2.0 * d) * (1.0 + 1e-12) / S.cell_s);
    if (!(need <= (double)RESCAN_MAX_REACH)) {
        atomicOr(v.flags, FLAG_SKIN);
        return RESCAN_MAX_REACH;
    }
    return (int)need > S.reach ? (int)need : S.reach;
}

// Visit the neighbours recorded in slot a's mask words, four at a time
// (positions and payloads, then compute). Bit k of word r is the k-th slot of
// cell row r of the block; r_ab = r_a - r_b is formed in FP64 exactly as in
// the scan. The skin mask also holds pairs out to R s: those that fail the
// exact predicate |r_ab|^2 < (2h)^2 are skipped (in FP32 contexts decided
// through the FP32 band of pair_within, with the same verdict).
template <typename T, int NB = 4, typename LoadFn, typename ComputeFn>
__device__ __forceinline__ void mask_neighbours(const EvalView<T>& v, const SysDev<T>& S, uint32_t a, double2 pa,
                                                const RowMask& M, LoadFn&& load, ComputeFn&& compute) {
    using P = typename std::decay<decltype(load(0u))>::type;
    const uint32_t ny = (uint32_t)S.ny;
    const uint32_t local = v.cell[a] - S.cell_base;
    const int cx = (int)(local / ny);
    const int cy = (int)(local - (uint32_t)cx * ny);
    const int R = S.reach;
    const int ylo = cy - R < 0 ? 0 : cy - R;
    const int xlo = cx - R < 0 ? 0 : cx - R;
    const int xhi = cx + R > S.nx - 1 ? S.nx - 1 : cx + R;
    // first slot of every row of the block (rows past the grid edge have no bits)
    uint32_t st[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        const int X = xlo + r;
        st[r] = X <= xhi ? v.cstart[S.cell_base + (uint32_t)X * ny + ylo] : 0u;
    }
    // queue of (word, first slot) of the non-empty rows, front in (m, base);
    // built once, so taking the next bit never has to skip an empty row
    uint32_t qm[5] = {0u, 0u, 0u, 0u, 0u}, qb[5] = {0u, 0u, 0u, 0u, 0u};
    int nq = 0;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
        // append row r when its word is non-empty (selects, no indexing)
        const bool put = M.w[r] != 0u;
#pragma unroll
        for (int i = 0; i <= r; ++i) {
            const bool here = put && nq == i;
            qm[i] = here ? M.w[r] : qm[i];
            qb[i] = here ? st[r] : qb[i];
        }
        nq += put ? 1 : 0;
    }
    uint32_t m = qm[0], base = qb[0];
    uint32_t m1 = qm[1], b1 = qb[1], m2 = qm[2], b2 = qb[2], m3 = qm[3], b3 = qb[3], m4 = qm[4], b4 = qb[4];
    const float r2_in = S.r2_in, r2_out = S.r2_out;
    const double R2 = S.R2;
    // next recorded neighbour; false once every word is spent
    auto next = [&](uint32_t& b) -> bool {
        const bool ok = m != 0u;
        b = ok ? base + (uint32_t)__builtin_ctz(m) : a;
        m &= m - 1u;
        const bool adv = m == 0u;
        m = adv ? m1 : m;
        base = adv ? b1 : base;
        m1 = adv ? m2 : m1;
        b1 = adv ? b2 : b1;
        m2 = adv ? m3 : m2;
        b2 = adv ? b3 : b2;
        m3 = adv ? m4 : m3;
        b3 = adv ? b4 : b3;
        m4 = adv ? 0u : m4;
        return ok;
    };
    while (true) {
        uint32_t bb[NB];
        bool ok[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) ok[j] = next(bb[j]);
        if (!ok[0]) break;
        double2 q[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) q[j] = at(v.pos, bb[j]);
        // payloads unconditionally: a spent lane's index is its own slot, so
        // every load is in bounds and none needs a branch around it
        P pl[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) pl[j] = load(bb[j]);
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (ok[j]) {
                const double ex = pa.x - q[j].x, ey = pa.y - q[j].y;
                const T dx = (T)ex, dy = (T)ey;
                const T r2w = dx * dx + dy * dy;   // the sweeps form the same square
                bool in;
                if constexpr (sizeof(T) == 4) {
                    in = pair_within(ex, ey, r2w, r2_in, r2_out, R2);
                } else {
                    double fx, fy;
                    in = pair_r2(pa, q[j], fx, fy) < R2;
                }
                if (in) compute(bb[j], dx, dy, pl[j]);
            }
        }
    }
}

__device__ __forceinline__ RowMask load_mask(const uint4* nmask, const uint32_t* nmask4, uint32_t a) {
    const uint4 w = nmask[a];
    RowMask M;
    M.w[0] = w.x;
    M.w[1] = w.y;
    M.w[2] = w.z;
    M.w[3] = w.w;
    M.w[4] = nmask4[a];
    return M;
}

// The neighbours of slot a: from its mask, or by scanning its cells when it
// had more candidates than the mask holds.
// RESCAN: the half step of slot a's system outran the skin mask; the
// step-start cells are scanned with reach `rescan` instead (the kernels built
// with RESCAN run only for such systems, so the others keep their registers).
// keep: the mask bits this lane visits (several lanes can share slot a, each
// visiting its own bits of every cell row); scans: whether this lane scans the
// cells when there is no mask to split (an overflowed mask, a rescan).
template <typename T, int NB = 4, bool RESCAN = false, typename LoadFn, typename ComputeFn>
__device__ __forceinline__ void neighbours(const EvalView<T>& v, const SysDev<T>& S, uint32_t a, double2 pa,
                                           LoadFn&& load, ComputeFn&& compute, int rescan = 0, uint32_t keep = ~0u,
                                           bool scans = true) {
    if constexpr (RESCAN) {
        if (scans) scan_cells<T, 1>(S, v.cstart, v.cell[a], a, pa, v.pos, load, compute, rescan);
    } else {
        RowMask M = load_mask(v.nmask, v.nmask4, a);
        if (!(M.w[4] & MASK_OVERFLOW)) {
#pragma unroll
            for (int r = 0; r < 5; ++r) M.w[r] &= keep;
            mask_neighbours<T, NB>(v, S, a, pa, M, load, compute);
        } else if (scans) {
            scan_cells<T, 1>(S, v.cstart, v.cell[a], a, pa, v.pos, load, compute, S.reach);  // rare: keep it lean
        }
    }
}

// Half step: whether system sys outran the skin mask (its sweeps then run in
// the RESCAN kernels); false in the first evaluation of a step.
template <typename T>
__device__ __forceinline__ bool outran(const EvalView<T>& v, int sys) {
    return v.skin_max != nullptr && v.skin_max[sys] != 0ull;
}

// The system of sweep chunk c (one 64-slot wave chunk of one system).
template <typename T>
__device__ __forceinline__ int chunk_system(const EvalView<T>& v, uint32_t c) {
    int lo = 0, hi = v.n_sys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (v.chunk_base[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    return __builtin_amdgcn_readfirstlane(lo);
}

// Grid of the RESCAN kernels: its waves stride over the chunks of the systems
// that outran the skin mask; with none (skin_max[n_sys], the largest over all
// systems, is 0) every wave returns at once. The half step's surface sweep
// carries as many workgroups past its own grid for the same systems' entries.
constexpr int RESCAN_BLOCKS = 256;

template <typename T, typename Fn>
__device__ __forceinline__ void for_outran_chunks(const EvalView<T>& v, Fn&& body) {
    if (v.skin_max[v.n_sys] == 0ull) return;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t waves = gridDim.x * wpb;
    const uint32_t total = v.chunk_base[v.n_sys];
    for (uint32_t c = blockIdx.x * wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); c < total; c += waves) {
        const int sys = chunk_system(v, c);
        if (v.skin_max[sys] == 0ull) continue;
        const uint32_t a = v.sys_lo[sys] + (c - v.chunk_base[sys]) * 64u + (uint32_t)__lane_id();
        body(sys, a, c, __builtin_amdgcn_readfirstlane(rescan_reach(v, v.sys[sys], sys)));
    }
}

template <typename T> struct Pay2 { V2<T> vel; V4<T> eos; };
template <typename T> struct Pay3 { V2<T> nrm; T vol; };

// Repulsive-force walls (eq. 29): the force per unit mass on every fluid
// particle of a system with boundary = 1, f = n R(psi) P(xi) eps(z, u_perp)
// summed over the system's wall and piston particles within reach, in FP64.
// The paper names R, P and eps without defining them; the published forms of
// the references it cites are used (psi = (r_a - r_k) . n_k, xi the distance
// along the wall):
//   R = 0.01 c_a^2 / h (1 - q) / sqrt(q), q = psi / (2h), for 0 < psi < 2h;
//   P = (1 + cos(pi xi / db)) / 2 for xi < db, db the wall-particle spacing (the
//       P of equally spaced wall particles sum to 1 along a straight wall);
//   eps = 1 + min(|20 u_perp| / c0, 1) when u_perp = (v_a - v_k) . n_k < 0, else 1
//       (no still-water depth: the depth term is taken as 1).
// Walls and pistons sit in two static cell grids per system (cells of
// 2h + db, so a 3 x 3 block covers the reach); a piston moves rigidly, so its
// records are looked up at the fluid particle's position less the piston's
// travel since the grids were built.
template <typename T>
__global__ void __launch_bounds__(256) k_wall_force(EvalView<T> v, WallView W) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= v.n) return;
    const uint32_t t = v.tag[a];
    if (tag_type(t) != T_FLUID) return;
    const int sys = (int)tag_sys(t);
    const SysDev<T>& S = v.sys[sys];
    if (!S.boundary) return;
    const WallSys& G = W.sys[sys];
    const double2 pa = v.pos[a];
    const V2<T> va = v.vel[a];
    const double rho = S.rho0_64 + (double)v.dens[a];
    const double r3 = rho / S.rho0_64;
    const double c = S.gamma7 ? (double)S.c0 * r3 * r3 * r3 : (double)S.c0 * pow(r3, (double)S.half_gm1);
    const double A = 0.01 * c * c / S.h64;
    const double two_h = 2.0 * S.h64;
    // the evaluation's time: the piston's travel and speed at it
    const double tm = W.time[sys] + (W.half ? 0.5 * W.dt[sys] : 0.0);
    const double X = S.pomega == 0.0 ? S.pu * tm : S.pu * (tm + S.pamp * (1.0 - cos(S.pomega * tm)) / S.pomega);
    const double U = S.pu * (1.0 + S.pamp * sin(S.pomega * tm));
    double fx = 0.0, fy = 0.0;
    for (int g = 0; g < 2; ++g) {
        const double sx = g ? (X - G.x_ref) * S.pdx : 0.0, sy = g ? (X - G.x_ref) * S.pdy : 0.0;
        const double ux = g ? U * S.pdx : 0.0, uy = g ? U * S.pdy : 0.0;
        const double qx = pa.x - sx, qy = pa.y - sy;   // in the grid's frame
        const int cx = (int)floor((qx - G.x0) * G.inv_cs), cy = (int)floor((qy - G.y0) * G.inv_cs);
        for (int X2 = cx - 1; X2 <= cx + 1; ++X2) {
            if (X2 < 0 || X2 >= G.nx) continue;
            const uint32_t row = G.cell_base[g] + (uint32_t)X2 * (uint32_t)G.ny;
            const int y0 = cy - 1 < 0 ? 0 : cy - 1, y1 = cy + 1 > G.ny - 1 ? G.ny - 1 : cy + 1;
            if (y0 > y1) continue;
            for (uint32_t k = W.cstart[row + y0]; k < W.cstart[row + y1 + 1]; ++k) {
                const double4 w = W.rec[k];   // position in the grid's frame, unit normal
                const double dx = qx - w.x, dy = qy - w.y;
                const double psi = dx * w.z + dy * w.w;
                if (!(psi > 0.0 && psi < two_h)) continue;
                const double tx = dx - psi * w.z, ty = dy - psi * w.w;
                const double xi = sqrt(tx * tx + ty * ty);
                if (!(xi < G.db)) continue;
                const double q = psi / two_h;
                const double R = A * (1.0 - q) / sqrt(q);
                const double P = 0.5 * (1.0 + cos(3.14159265358979323846 * xi / G.db));
                const double up = ((double)va.x - ux) * w.z + ((double)va.y - uy) * w.w;
                const double eu = up >= 0.0 ? 0.0 : fmin(fabs(20.0 * up) / (double)S.c0, 1.0);
                const double f = R * P * (1.0 + eu);
                fx += f * w.z;
                fy += f * w.w;
            }
        }
    }
    V2<T> out;
    out.x = (T)fx;
    out.y = (T)fy;
    v.fwall[a] = out;
}

// Density summation (eq. 6) for the fluid particles of systems that use it:
// rho_a = sum_b m_b W_ab over every active particle of the system, itself
// included, summed in FP64 whatever the storage type -- the stored rho - rho0
// keeps the Tait pressure's precision only if the sum is exact to well below
// an FP32 ulp of rho0 -- and written, with m / rho, to the evaluation's
// state before the colour sweep reads m_b / rho_b. The cells are scanned with
// the exact pair predicate: the step-start cells in the half step too, with
// the rescan reach where the system outran the skin.
template <typename T>
__global__ void __launch_bounds__(256) k_density(EvalView<T> v) {
    int sys;
    uint32_t a;
    if (!wave_assign(v, sys, a)) return;
    const SysDev<T>& S = v.sys[sys];
    if (!S.density_sum) return;
    const int rr = v.skin_max ? rescan_reach(v, S, sys) : 0;
    const int R = __builtin_amdgcn_readfirstlane(rr ? rr : S.reach);
    if (a >= v.sys_hi[sys] || tag_type(v.tag[a]) != T_FLUID) return;
    const double inv_h = 1.0 / S.h64;
    const double m_a = (double)v.mass[a];
    double sum = m_a;   // the self term m_a W(0), W(0) = wnorm
    scan_cells_rows<T>(S, v.cstart, v.cell[a], a, v.pos[a], v.pos, [&](uint32_t b) { return v.mass[b]; },
                       [&](uint32_t, uint32_t, T, T, double r2, T m_b) {
                           sum += (double)m_b * kernel_shape64(S.kernel, sqrt(r2) * inv_h);
                       },
                       [](int) {}, S.R2, R);
    const double rho = S.wnorm64 * sum;
    v.dens_out[a] = (T)(rho - S.rho0_64);
    v.vol_out[a] = (T)(m_a / rho);
}

// Sweep 1: colour function C_a = sum_b (m_b / rho_b) W_ab, self included
// (eq. 14). The Tait equation (eq. 26) is evaluated here once per particle:
// the record (P / rho^2, C, rho, +-m / rho) is everything the main sweep
// gathers of a neighbour besides its position and velocity (the sound speed
// follows from rho; m / rho carries a minus sign for a boundary particle, so
// the sweep needs no type tag of its neighbours).
//
// The first evaluation of a step scans the cells. Its candidates within R s
// (the cell block's radius) are recorded as the skin mask, and those within 2h
// enter the colour sum. Every other sweep of the step walks the skin mask with
// the exact pair predicate: the first evaluation's main and surface sweeps,
// and the whole half-step evaluation (k_colour_skin first), since the predictor
// keeps every particle within half the skin of its step-start position, so
// every pair within 2h at the half step is in it. The walk visits the pairs
// within 2h in the order a scan would.
// Eight waves per SIMD (at most 64 VGPRs): the candidate scan is issue-bound
// and hides its gathers best with the most waves (measured 5% faster than 7).

// Mask words under construction: `cur` collects the row being scanned,
// row_end files it.
struct MaskBuilder {
    RowMask M = {{0u, 0u, 0u, 0u, 0u}};
    uint32_t cur = 0;
    bool overflow = false;
    __device__ void mark(uint32_t k) {
        if (k < MASK_ROW_BITS) cur |= 1u << k;
        else overflow = true;
    }
    __device__ void row_end(int r) {
        M.w[0] = r == 0 ? cur : M.w[0];
        M.w[1] = r == 1 ? cur : M.w[1];
        M.w[2] = r == 2 ? cur : M.w[2];
        M.w[3] = r == 3 ? cur : M.w[3];
        M.w[4] = r == 4 ? cur : M.w[4];
        cur = 0;
    }
    // bit 31 of the last word is the overflow flag, so that row holds 31 bits
    __device__ void store(uint4* w03, uint32_t* w4, uint32_t a) {
        if (M.w[4] & MASK_OVERFLOW) overflow = true;
        w03[a] = make_uint4(M.w[0], M.w[1], M.w[2], M.w[3]);
        w4[a] = overflow ? (M.w[4] | MASK_OVERFLOW) : M.w[4];
    }
};

// The colour, then the record of slot a.
template <typename T>
__device__ __forceinline__ void colour_finish(const EvalView<T>& v, const SysDev<T>& S, uint32_t a, T vol_a,
                                              T dens_a, T wsum, bool fluid_a) {
    const T sum = vol_a * S.W0 + S.wnorm * wsum;
    v.colour[a] = sum;
    T rho_a, pr_a;
    tait(S, dens_a, rho_a, pr_a);
    V4<T> e;
    e.x = pr_a;
    e.y = sum;
    e.z = rho_a;
    e.w = fluid_a ? vol_a : -vol_a;   // the sign tells the main sweep a boundary particle
    v.eos[a] = e;
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_colour(EvalView<T> v) {
    int sys;
    uint32_t a;
    if (!wave_assign(v, sys, a)) return;
    const SysDev<T>& S = v.sys[sys];
    if (a >= v.sys_hi[sys]) return;
    const KernelConsts<T> K = kconsts(S);
    const double2 pa = v.pos[a];
    const T vol_a = v.vol[a];
    const T dens_a = v.dens[a];   // for the record written at the end
    const double R2 = S.R2;
    T wsum = 0;   // sum_b (m_b / rho_b) W_ab / wnorm
    MaskBuilder Sk;   // the skin mask: pairs within R s
    auto load = [&](uint32_t b) { return v.vol[b]; };
    auto acc = [&](uint32_t, T dx, T dy, T vol_b) { wsum += vol_b * kernel_shape(K, sqrt_(dx * dx + dy * dy)); };
    auto row_end = [&](int r) { Sk.row_end(r); };
    if (S.reach == 1) {
        // 3 x 3 blocks (about 3.5 candidates per neighbour): first the pair
        // predicates alone, recorded as the mask, then the kernel sum over the
        // mask, whose walk applies the exact predicate, so lanes do not pay for
        // each other's rejected candidates
        scan_cells_rows<T>(S, v.cstart, v.cell[a], a, pa, v.pos, [&](uint32_t) { return 0; },
                           [&](uint32_t, uint32_t k, T, T, double, int) { Sk.mark(k); }, row_end, S.Rs2, S.reach);
        if (!Sk.overflow) mask_neighbours<T>(v, S, a, pa, Sk.M, load, acc);
        else scan_cells<T>(S, v.cstart, v.cell[a], a, pa, v.pos, load, acc, S.reach);
    } else {
        // 5 x 5 blocks (about 2.2 candidates per neighbour): one pass
        scan_cells_rows<T>(S, v.cstart, v.cell[a], a, pa, v.pos, load,
                           [&](uint32_t, uint32_t k, T, T, double r2, T vol_b) {
                               Sk.mark(k);
                               if (r2 < R2) wsum += vol_b * kernel_shape(K, sqrt_((T)r2));
                           },
                           row_end, S.Rs2, S.reach);
    }
    colour_finish(v, S, a, vol_a, dens_a, wsum, tag_type(v.tag[a]) == T_FLUID);
    Sk.store(v.smask, v.smask4, a);
}

// Sweep 1 of the half-step evaluation: the same colour sum over the skin mask
// of the first evaluation (v.nmask), which the walk filters by the exact
// predicate; the sweeps that follow walk the same skin mask.
template <typename T, bool RESCAN>
__device__ __forceinline__ void colour_skin_slot(const EvalView<T>& v, int sys, uint32_t a, int rescan) {
    const SysDev<T>& S = v.sys[sys];
    const KernelConsts<T> K = kconsts(S);
    const double2 pa = v.pos[a];
    const T vol_a = v.vol[a];
    const T dens_a = v.dens[a];
    T wsum = 0;
    neighbours<T, 4, RESCAN>(v, S, a, pa, [&](uint32_t b) { return at(v.vol, b); },
                             [&](uint32_t, T dx, T dy, T vol_b) { wsum += vol_b * kernel_shape(K, sqrt_(dx * dx + dy * dy)); },
                             rescan);
    colour_finish(v, S, a, vol_a, dens_a, wsum, tag_type(v.tag[a]) == T_FLUID);
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) k_colour_skin(EvalView<T> v) {
    int sys;
    uint32_t a;
    if (!wave_assign(v, sys, a)) return;
    if (outran(v, sys)) return;   // k_colour_rescan
    if (a >= v.sys_hi[sys]) return;
    colour_skin_slot<T, false>(v, sys, a, 0);
}

// Its own kernel (not workgroups past the colour sweep's grid, as in the
// surface sweep): the colour sweep's code comes out slower with it.
template <typename T>
__global__ void __launch_bounds__(256) k_colour_rescan(EvalView<T> v) {
    for_outran_chunks(v, [&](int sys, uint32_t a, uint32_t, int rescan) {
        if (a < v.sys_hi[sys]) colour_skin_slot<T, true>(v, sys, a, rescan);
    });
}

// Sweep 2: continuity (eq. 7) for every active particle (a boundary particle
// sums over fluid neighbours only); for fluid particles also the pressure +
// artificial-viscosity acceleration (eq. 9-10) and the interface normal
// n_a = sum_b (m_b/rho_b)(C_b - C_a) grad_a W_ab (eq. 18); the signal term
// max_b |h v_ab . r_ab| / r_ab^2 feeds the eq. 31 limit.
// The normal filter N_a = [|n_a| > eps] (eq. 20-21) is applied here: a fluid
// particle that fails it has no surface force (kappa = 0: the curvature arrays
// hold values for filtered particles only), so its total acceleration (eq. 25,
// gravity added) and eq. 30 term are final; one that passes is appended to the
// surface list for k_surface. The list has SURF_REGIONS regions with a counter
// each: a wave appends to region (chunk / SURF_BLOCK) % SURF_REGIONS, so the
// waves running at one time spread their appends over the counters while a
// region collects neighbouring chunks (its neighbours share cache lines). The wave's minima of the two dt terms go
// to its own slot of dt_wave (plain stores); k_dt_finalize reduces them.
// FP32: six waves per SIMD (at most 80 VGPRs) fit without spilling.
// One wave's chunk of the main sweep (every lane of the wave calls it).
// RESCAN: the half step of a system that outran its skin mask scans the
// step-start cells with the wider reach `rescan`.
template <typename T, bool RESCAN>
__device__ __forceinline__ void main_chunk(const EvalView<T>& v, int sys, uint32_t a, uint32_t chunk, int rescan) {
    const SysDev<T>& S = v.sys[sys];
    const bool valid = a < v.sys_hi[sys];
    // the arguments of this particle's dt terms: c_a + v_sig (eq. 31) and, when
    // the sweep finishes the particle, |a| (eq. 30); 0 where there is none
    T cvs = 0, amf = 0;
    bool surf = false;
    if (valid) {
        const bool fluid = tag_type(v.tag[a]) == T_FLUID;
        const double2 pa = v.pos[a];
        const V2<T> va = v.vel[a];
        const V4<T> ea = v.eos[a];
        const T pr_a = ea.x, Ca = ea.y, rho_a = ea.z;
        const T c_a = sound_speed(S, rho_a);
        const T vc_a = -S.alpha_h * c_a;
        const T h = S.h, eta2 = S.eta2;
        const KernelConsts<T> K = kconsts(S);
        T drho = 0, ax = 0, ay = 0, nx = 0, ny = 0, sig_vr = 0, sig_r2 = 1;
        auto pair = [&](uint32_t, T dx, T dy, const Pay2<T>& p) {
                // the record's m/rho is negative for a boundary particle
                if (!fluid && !(p.eos.w > T(0))) return;
                const T pr_b = p.eos.x, C_b = p.eos.y, rho_b = p.eos.z, vol_b = fabs(p.eos.w);
                T r2 = dx * dx + dy * dy;
                T F = kernel_f(K, sqrt_(r2));
                T ux = va.x - p.vel.x, uy = va.y - p.vel.y;
                T vr = ux * dx + uy * dy;
                const T vF = vol_b * F;
                const T mF = vF * rho_b;   // m_b F
                drho += mF * vr;
                // signal term max_b |v_ab . r_ab| / r_ab^2, kept as a fraction
                const T avr = fabs(vr);
                const bool up = avr * sig_r2 > sig_vr * r2;
                sig_vr = up ? avr : sig_vr;
                sig_r2 = up ? r2 : sig_r2;
                if (fluid) {
                    T pi = 0;
                    if (vr < T(0)) {
                        // the mean sound speed over the mean density: the halves cancel
                        pi = (vc_a + visc_speed(S, rho_b)) * vr * rcp((rho_a + rho_b) * (r2 + eta2));
                    }
                    T coef = mF * (pr_a + pr_b + pi);
                    ax -= coef * dx;
                    ay -= coef * dy;
                    T cn = (C_b - Ca) * vF;
                    nx += cn * dx;
                    ny += cn * dy;
                }
            };
        auto global_load = [&](uint32_t b) {
            Pay2<T> p;
            p.vel = at(v.vel, b);
            p.eos = at(v.eos, b);
            return p;
        };
        neighbours<T, 4, RESCAN>(v, S, a, pa, global_load, pair, rescan);
        const T vsig = h * sig_vr / sig_r2;
        v.drho[a] = drho;
        V2<T> acc, nrm;
        nrm.x = nx;
        nrm.y = ny;
        v.nrm[a] = nrm;
        cvs = c_a + vsig;
        const T mag = sqrt_(nx * nx + ny * ny);
        surf = fluid && mag > S.eps;
        if (S.boundary && fluid) {   // repulsive-force walls (eq. 29), from k_wall_force
            const V2<T> fw = v.fwall[a];
            ax += fw.x;
            ay += fw.y;
        }
        if (fluid && !surf) {
            // no surface force: acceleration and curvature are final here
            const bool gon = gravity_on(S, pa);
            acc.x = ax + (gon ? S.gx : T(0));
            acc.y = ay + (gon ? S.gy : T(0));
            const T am = sqrt_(acc.x * acc.x + acc.y * acc.y);
            amf = am;
        } else {
            // filtered particles: k_surface adds the surface force and gravity
            acc.x = ax;
            acc.y = ay;
        }
        v.acc[a] = acc;
    }
    if (v.do_dt) {
        // h / (c + v_sig) and sqrt(h / |a|) fall as their arguments grow, after
        // rounding too, so the wave's smallest terms are those of its largest
        // arguments: one maximum each, then one division per wave (a NaN
        // argument fails > 0 and drops out, as it would from a minimum)
        const T m_cv = wave_max_nonneg(cvs > T(0) ? cvs : T(0));
        const T m_f = wave_max_nonneg(amf > T(0) ? amf : T(0));
        if (__lane_id() == 0) {
            const T h = S.h;
            v.dt_wave[2 * (size_t)chunk] = m_cv > T(0) ? (double)(h / m_cv) : __builtin_inf();
            v.dt_wave[2 * (size_t)chunk + 1] = m_f > T(0) ? sqrt((double)S.h / (double)m_f) : __builtin_inf();
        }
    }
    const unsigned long long bal = __ballot(surf);
    if (bal) {
        const uint32_t r = (chunk / SURF_BLOCK) % SURF_REGIONS;
        const int first = __ffsll((long long)bal) - 1;
        uint32_t base = 0;
        if (__lane_id() == first) base = atomicAdd(v.surf_count + r, (uint32_t)__popcll(bal));
        base = __shfl(base, first, 64);
        if (surf) {
            const uint32_t idx = base + (uint32_t)__popcll(bal & ((1ull << __lane_id()) - 1ull));
            if (idx < v.surf_region) v.surf_list[(size_t)r * v.surf_region + idx] = a;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 6 : 1))) k_main(EvalView<T> v) {
    int sys;
    uint32_t a, chunk;
    if (!wave_assign(v, sys, a, &chunk)) return;
    if (outran(v, sys)) return;   // k_main_rescan
    main_chunk<T, false>(v, sys, a, chunk, 0);
}

// Its own kernel (not workgroups past the main sweep's grid, as in the surface
// sweep): inside the main sweep the rescan's registers would spill.
template <typename T>
__global__ void __launch_bounds__(256) k_main_rescan(EvalView<T> v) {
    for_outran_chunks(v, [&](int sys, uint32_t a, uint32_t chunk, int rescan) {
        main_chunk<T, true>(v, sys, a, chunk, rescan);
    });
}

// Sweep 3, over the surface list (fluid particles with N_a = 1): curvature
// kappa_a = sum_b min(N_a,N_b)(m_b/rho_b)(nh_b - nh_a).grad_a W_ab /
// sum_b min(N_a,N_b)(m_b/rho_b) W_ab (eq. 23, self in the denominator),
// surface-tension acceleration -(sigma/rho_a) kappa_a n_a (eq. 24) and the
// total acceleration (eq. 25); |a| feeds the eq. 30 limit. Boundary particles
// carry n = 0, so they fail the filter and drop out of both sums.
// The list holds a few percent of the particles, from every system, so the
// waves here are dense but not system-uniform: the system's constants are
// per lane. A fixed grid strides over the regions, taken as one list.
// RESCAN: the entries of systems whose half step outran the skin mask (and
// only those; the plain kernel skips them).
template <typename T, bool RESCAN>
__device__ __forceinline__ void surface_pass(const EvalView<T>& v, uint32_t blk, uint32_t nblk) {
    if (RESCAN && (v.skin_max == nullptr || v.skin_max[v.n_sys] == 0ull)) return;
    __shared__ uint32_t pre[4][SURF_REGIONS];
    static_assert(SURF_REGIONS == 64, "one region per lane");
    const int lane = __lane_id(), w = (int)(threadIdx.x >> 6);
    // exclusive prefix of the region counts (one per lane), kept in LDS so the
    // entries below can look it up from divergent code
    const uint32_t cnt = v.surf_count[lane] < v.surf_region ? v.surf_count[lane] : v.surf_region;
    uint32_t incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(incl, o, 64);
        if (lane >= o) incl += y;
    }
    pre[w][lane] = incl - cnt;
    const uint32_t total = __shfl(incl, 63, 64);
    __shared__ uint32_t cl_n[4], cl_base;
    __syncthreads();
    // A short list (at most SURF_SPLIT_MAX entries) gives each entry four
    // adjacent lanes, which split its neighbours by mask bit (sub = the lane's
    // place among them): its chain of dependent loads is shorter and the chip
    // gets more waves. A long list already fills the chip: one lane per entry.
    // The workgroup takes 256 / G consecutive entries per pass, so all its
    // waves run the same passes and can share the closure-list atomic.
    const int G = total <= SURF_SPLIT_MAX ? 4 : 1;   // the same in every wave
    const int sub = lane & (G - 1);
    const uint32_t keep = G == 4 ? 0x11111111u << sub : ~0u;
    const uint32_t per_block = blockDim.x / (uint32_t)G, per_wave = 64u / (uint32_t)G;
    for (uint32_t e0 = blk * per_block; e0 < total; e0 += nblk * per_block) {
        const uint32_t e = e0 + (uint32_t)w * per_wave;
        const uint32_t idx = e + (uint32_t)(lane >> (G == 4 ? 2 : 0));
        // region holding entry idx: the last r with pre[r] <= idx
        int r = 0;
#pragma unroll
        for (int step = 32; step > 0; step >>= 1)
            if (pre[w][r + step] <= idx) r += step;
        const uint32_t off = idx - pre[w][r];
        // the same for the G lanes of an entry
        bool in = idx < total && off < v.surf_region;
        const uint32_t a = in ? v.surf_list[(size_t)r * v.surf_region + off] : 0u;
        const uint32_t sys = in ? tag_sys(v.tag[a]) : 0u;
        in = in && (RESCAN ? outran(v, (int)sys) : !outran(v, (int)sys));
        const SysDev<T>& S = v.sys[sys];
        T num = 0, den = 0;   // this lane's share of the two sums
        if (in) {
            const T eps = S.eps;
            const KernelConsts<T> K = kconsts(S);
            const V2<T> n_a = v.nrm[a];
            const T im = rcp(sqrt_(n_a.x * n_a.x + n_a.y * n_a.y));
            const T hx = n_a.x * im, hy = n_a.y * im;
            neighbours<T, 4, RESCAN>(v, S, a, v.pos[a],
                [&](uint32_t b) { return Pay3<T>{at(v.nrm, b), at(v.vol, b)}; },
                [&](uint32_t, T dx, T dy, const Pay3<T>& p) {
                    T mb = sqrt_(p.nrm.x * p.nrm.x + p.nrm.y * p.nrm.y);
                    if (mb > eps) {
                        T ib = rcp(mb);
                        T rr = sqrt_(dx * dx + dy * dy);
                        T W, F;
                        kernel_wf(K, rr, W, F);
                        num += p.vol * F * ((p.nrm.x * ib - hx) * dx + (p.nrm.y * ib - hy) * dy);
                        den += p.vol * W;
                    }
                },
                RESCAN ? rescan_reach(v, S, (int)sys) : 0, keep, sub == 0);
        }
        if (G == 4) {
            // the entry's sums over its four lanes (every lane of the wave is
            // active here, and an entry's lanes are adjacent)
#pragma unroll
            for (int o = 1; o < 4; o <<= 1) {
                num += __shfl_xor(num, o, 64);
                den += __shfl_xor(den, o, 64);
            }
        }
        const bool lead = in && sub == 0;
        double dtf = __builtin_inf();
        bool listed = false;
        if (lead) {
            const V2<T> n_a = v.nrm[a];
            V2<T> acc = v.acc[a];
            const T rho_a = v.eos[a].z;
            const double2 pa = v.pos[a];
            // with the learned closure the surface force of a filtered particle is
            // added later, from the network's curvature or the plain fallback
            listed = v.cl_count != nullptr && S.closure != 0;
            den += v.vol[a] * S.W0;   // self term of the denominator
            const T kappa = num / den;
            v.kappa_plain[a] = kappa;
            T f = listed ? T(0) : -S.sigma * rcp(rho_a) * kappa;
            const bool gon = gravity_on(S, pa);
            acc.x += f * n_a.x + (gon ? S.gx : T(0));
            acc.y += f * n_a.y + (gon ? S.gy : T(0));
            v.acc[a] = acc;
            v.kappa[a] = kappa;
            T am = sqrt_(acc.x * acc.x + acc.y * acc.y);
            if (am > T(0) && !listed) dtf = sqrt((double)S.h / (double)am);
        }
        if (v.do_dt) atomic_min_per_system(v.dtmin + 1, 2, (int)sys, dtf, lead);
        if (v.cl_count) {
            // append the listed slots, one atomic per workgroup and pass
            const unsigned long long bal = __ballot(listed);
            if (lane == 0) cl_n[w] = (uint32_t)__popcll(bal);
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t tot = cl_n[0] + cl_n[1] + cl_n[2] + cl_n[3];
                cl_base = tot ? atomicAdd(v.cl_count, tot) : 0u;
            }
            __syncthreads();
            if (listed) {
                uint32_t ci = cl_base + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
                for (int k = 0; k < w; ++k) ci += cl_n[k];
                if (ci < v.cl_capacity) v.cl_list[ci] = a;
            }
            __syncthreads();
        }
    }
}

// The first sweep_blocks workgroups take the entries of the systems that kept
// to their skin masks; any past them, those of the systems that outran theirs.
template <typename T>
__global__ void __launch_bounds__(256) k_surface(EvalView<T> v, unsigned sweep_blocks) {
    if (blockIdx.x < sweep_blocks) surface_pass<T, false>(v, blockIdx.x, sweep_blocks);
    else surface_pass<T, true>(v, blockIdx.x - sweep_blocks, gridDim.x - sweep_blocks);
}

// ------------------------------------------------------------------ time step

// dt of every system (eq. 32): the minima of h/(c + sig) (eq. 31) and
// sqrt(h/|a|) (eq. 30) over the per-wave minima of the main sweep (dt_wave,
// one pair per chunk of the system) and what the surface and closure kernels
// folded into dtmin; dtmin is reset for the next step, and the system's largest
// half-step displacement for this step's predictor. One workgroup per system.
template <typename T>
__global__ void __launch_bounds__(1024) k_dt_finalize(int n_sys, const SysDev<T>* sys, const uint32_t* chunk_base,
                                                     const double* dt_wave, unsigned long long* dtmin, double* dt,
                                                     unsigned long long* skin_max) {
    __shared__ double red[2][16];
    const int s = blockIdx.x;
    if (s >= n_sys) return;
    const uint32_t c0 = chunk_base[s], c1 = chunk_base[s + 1];
    double cv = __builtin_inf(), f = __builtin_inf();
    for (uint32_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) {
        cv = fmin(cv, dt_wave[2 * (size_t)c]);
        f = fmin(f, dt_wave[2 * (size_t)c + 1]);
    }
    cv = wave_min(cv);
    f = wave_min(f);
    const int w = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        red[0][w] = cv;
        red[1][w] = f;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) {
            cv = fmin(cv, red[0][k]);
            f = fmin(f, red[1][k]);
        }
        const SysDev<T>& S = sys[s];
        f = fmin(f, __longlong_as_double((long long)dtmin[2 * s + 1]));   // sqrt(h/|a|)
        cv = fmin(cv, __longlong_as_double((long long)dtmin[2 * s + 0]));  // h/(c + sig)
        double d = S.dt_fixed > 0.0 ? S.dt_fixed : S.courant * fmin(f, cv);
        if (!(d < __builtin_inf())) d = 0.0;
        dt[s] = d;
        const unsigned long long inf_bits = (unsigned long long)__double_as_longlong(__builtin_inf());
        dtmin[2 * s] = inf_bits;
        dtmin[2 * s + 1] = inf_bits;
        skin_max[s] = 0ull;   // this step's predictor records its displacements afresh
        if (s == 0) skin_max[n_sys] = 0ull;
    }
}

__device__ __forceinline__ double piston_travel(double U, double A, double w, double t) {
    if (w == 0.0) return U * t;
    return U * (t + A * (1.0 - cos(w * t)) / w);
}
__device__ __forceinline__ double piston_speed(double U, double A, double w, double t) {
    return U * (1.0 + A * sin(w * t));
}

// A half-step displacement beyond half the cell skin: the system's largest one
// is kept (as the bit pattern of its square, whose unsigned order is the
// numeric order), so the half-step sweeps of that system scan the cells again
// with a reach that covers it. Rare; a NaN displacement fails the test and is
// caught as a non-finite value by the corrector.
template <typename T>
__device__ __forceinline__ void note_displacement(const IntegView<T>& v, const SysDev<T>& S, uint32_t sys, double dx,
                                                  double dy) {
    const double d2 = dx * dx + dy * dy;
    if (d2 > S.skin2) {
        const unsigned long long bits = (unsigned long long)__double_as_longlong(d2);
        atomicMax(v.skin_max + sys, bits);
        atomicMax(v.skin_max + v.n_sys, bits);   // the largest over all systems
        atomicOr(v.flags, FLAG_RESCAN);
    }
}

// Predictor: half-step state from state n and its derivatives.
template <typename T>
__global__ void k_predict(IntegView<T> v) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < SURF_REGIONS) v.surf_count[threadIdx.x] = 0u;   // the half step's list
    if (a >= v.n) return;
    uint32_t t = v.tag[a];
    uint32_t ty = tag_type(t);
    if (ty == T_INACTIVE) return;
    const SysDev<T>& S = v.sys[tag_sys(t)];
    double dt = v.dt[tag_sys(t)];
    double hd = 0.5 * dt;
    T hdt = (T)hd;
    double2 p = v.pos[a];
    V2<T> u = v.vel[a];
    // a summed density (eq. 6) is recomputed by the half-step evaluation; a
    // repulsive-force wall's density does not evolve
    const bool frozen = (ty == T_FLUID && S.density_sum) || (ty != T_FLUID && S.boundary);
    T dh = frozen ? v.dens[a] : v.dens[a] + hdt * v.drho[a];
    if (ty != T_FLUID && dh < T(0)) dh = T(0);   // boundaries never below rho0: they only repel
    v.dens_h[a] = dh;
    v.vol[a] = particle_vol(S, dh, v.mass[a]);
    if (ty == T_FLUID) {
        V2<T> acc = v.acc[a];
        double2 q;
        q.x = p.x + hd * (double)u.x;
        q.y = p.y + hd * (double)u.y;
        note_displacement(v, S, tag_sys(t), q.x - p.x, q.y - p.y);
        v.pos_h[a] = q;
        V2<T> w;
        w.x = u.x + hdt * acc.x;
        w.y = u.y + hdt * acc.y;
        v.vel_h[a] = w;
    } else if (ty == T_PISTON) {
        double tn = v.time[tag_sys(t)];
        double dX = piston_travel(S.pu, S.pamp, S.pomega, tn + hd) - piston_travel(S.pu, S.pamp, S.pomega, tn);
        double U = piston_speed(S.pu, S.pamp, S.pomega, tn + hd);
        double2 q;
        q.x = p.x + S.pdx * dX;
        q.y = p.y + S.pdy * dX;
        note_displacement(v, S, tag_sys(t), q.x - p.x, q.y - p.y);
        v.pos_h[a] = q;
        V2<T> w;
        w.x = (T)(S.pdx * U);
        w.y = (T)(S.pdy * U);
        v.vel_h[a] = w;
    } else {
        v.pos_h[a] = p;
        v.vel_h[a] = u;
    }
}

// Corrector: state n+1 from state n and the half-step derivatives, in place;
// fluid leaving the box becomes inactive; instability checks. With v.key set
// it also does the next sort's first pass on the new state (cell keys, slots
// within the cells, counts), in the key kernel's launch shape.
template <typename T>
__global__ void k_correct(IntegView<T> v) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = a < v.n;
    // the slot's state with its tag: the loads do not wait for the type test
    uint32_t t = valid ? v.tag[a] : 0u;
    double2 p = valid ? v.pos[a] : make_double2(0.0, 0.0);
    const uint32_t ty = tag_type(t);
    if (valid && ty != T_INACTIVE) {
        V2<T> u = v.vel[a];
        const V2<T> acc = v.acc[a];
        const T dens0 = v.dens[a], drho = v.drho[a];
        const SysDev<T>& S = v.sys[tag_sys(t)];
        double dt = v.dt[tag_sys(t)];
        T tdt = (T)dt;
        // eq. 6: the density of the half-step evaluation; eq. 7 otherwise
        const bool summed = ty == T_FLUID && S.density_sum;
        const bool wall_f = ty != T_FLUID && S.boundary;   // repulsive-force wall: density fixed
        T dens = summed ? v.dens_h[a] : (wall_f ? dens0 : dens0 + tdt * drho);
        if (ty != T_FLUID && dens < T(0)) dens = T(0);   // boundaries never below rho0
        v.dens[a] = dens;
        uint32_t flags = 0;
        if (!isfinite(dens)) flags |= FLAG_NONFINITE;
        else if (!wall_f && ((!summed && dens < T(-0.5) * S.rho0) || dens > S.rho0)) flags |= FLAG_DENSITY;
        if (ty == T_FLUID) {
            p.x = p.x + dt * ((double)u.x + 0.5 * dt * (double)acc.x);
            p.y = p.y + dt * ((double)u.y + 0.5 * dt * (double)acc.y);
            u.x += tdt * acc.x;
            u.y += tdt * acc.y;
            v.pos[a] = p;
            v.vel[a] = u;
            if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(u.x) || !isfinite(u.y)) flags |= FLAG_NONFINITE;
            if (p.x < S.box_lo_x || p.x > S.box_hi_x || p.y < S.box_lo_y || p.y > S.box_hi_y) {
                t = (t & ~15u) | T_INACTIVE;
                v.tag[a] = t;
            }
        } else if (ty == T_PISTON) {
            double tn = v.time[tag_sys(t)];
            double dX = piston_travel(S.pu, S.pamp, S.pomega, tn + dt) - piston_travel(S.pu, S.pamp, S.pomega, tn);
            double U = piston_speed(S.pu, S.pamp, S.pomega, tn + dt);
            p.x += S.pdx * dX;
            p.y += S.pdy * dX;
            v.pos[a] = p;
            V2<T> w;
            w.x = (T)(S.pdx * U);
            w.y = (T)(S.pdy * U);
            v.vel[a] = w;
        }
        if (flags) atomicOr(v.flags, flags);
    }
    if (v.key) key_and_count<T>(v.sys, a, valid, t, p, v.key, v.kslot, v.kcount, v.trash, v.kblk);
}

__global__ void k_advance_time(int n_sys, const double* dt, double* time) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < n_sys) time[s] += dt[s];
}

// ------------------------------------------------------------------ debug: neighbour lists
// The neighbours the sweeps visit, read back: after a sort and the first
// colour sweep (which records the skin mask), every slot's neighbours are
// walked exactly as the main and surface sweeps walk them -- the mask's
// candidates filtered by the exact pair predicate, or the cell scan where the
// mask overflowed.

template <typename T>
__global__ void k_nbr_count(EvalView<T> v, uint32_t* count) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= v.n) return;
    uint32_t t = v.tag[a];
    uint32_t c = 0;
    if (tag_type(t) != T_INACTIVE) {
        const SysDev<T>& S = v.sys[tag_sys(t)];
        neighbours<T, 1>(v, S, (uint32_t)a, v.pos[a], [](uint32_t) { return 0; },
                         [&](uint32_t, T, T, int) { ++c; });
    }
    count[a] = c;
}

template <typename T>
__global__ void k_nbr_fill(EvalView<T> v, int a0, int a1, const int64_t* start, int64_t base, uint32_t* out) {
    int a = a0 + blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= a1) return;
    uint32_t t = v.tag[a];
    if (tag_type(t) == T_INACTIVE) return;
    const SysDev<T>& S = v.sys[tag_sys(t)];
    int64_t k = start[a] - base;
    neighbours<T, 1>(v, S, (uint32_t)a, v.pos[a], [](uint32_t) { return 0; },
                     [&](uint32_t b, T, T, int) { out[k++] = v.id[b]; });
}

// ------------------------------------------------------------------ breakup length
// The breakup criterion of Section 3-2: the jet is broken where two fluid
// particles consecutive along its axis, beyond the nozzle exit, are more than
// the gap (1.5 h) apart. The coordinates xi = p . axis are binned in bins of
// half the gap: a larger gap always leaves a bin empty between its two ends,
// and no gap inside a bin can exceed it, so the consecutive pairs that matter
// are the maximum of a non-empty bin and the minimum of the next non-empty
// one -- the same values a sort would put side by side. FP64 coordinates go
// through an order-preserving map to 64-bit integers for the atomic extrema.

__device__ __forceinline__ unsigned long long ordered_bits(double x) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ __forceinline__ double from_ordered(unsigned long long k) {
    const unsigned long long u = (k >> 63) ? (k & 0x7FFFFFFFFFFFFFFFull) : ~k;
    return __longlong_as_double((long long)u);
}

// The coordinate along the axis (no FMA, as the oracle forms it).
__device__ __forceinline__ double axis_coord(double2 p, double ax, double ay) {
#pragma clang fp contract(off)
    return p.x * ax + p.y * ay;
}

// Per system: the largest coordinate of its fluid particles at or beyond the start.
template <typename T>
__global__ void k_breakup_extent(int n, const uint32_t* tag, const double2* pos, double ax, double ay,
                                 const double* start, unsigned long long* extent) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const uint32_t t = tag[a];
    if (tag_type(t) != T_FLUID) return;
    const double xi = axis_coord(pos[a], ax, ay);
    if (xi >= start[tag_sys(t)]) atomicMax(extent + tag_sys(t), ordered_bits(xi));
}

// Per bin of half the gap: the smallest and largest coordinate in it.
template <typename T>
__global__ void k_breakup_bins(int n, const uint32_t* tag, const double2* pos, double ax, double ay, const double* start,
                               const double* anchor, const double* half_gap, const uint32_t* bin_base,
                               unsigned long long* bmin, unsigned long long* bmax) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    const uint32_t t = tag[a];
    if (tag_type(t) != T_FLUID) return;
    const uint32_t s = tag_sys(t);
    const double xi = axis_coord(pos[a], ax, ay);
    if (!(xi >= start[s])) return;
    // bins counted from the anchor (the start, or the box's near edge beyond it)
    const double u = floor((xi - anchor[s]) / half_gap[s]);
    const uint32_t b = bin_base[s] + (uint32_t)(u > 0.0 ? u : 0.0);
    atomicMin(bmin + b, ordered_bits(xi));
    atomicMax(bmax + b, ordered_bits(xi));
}

// One workgroup per system: the first non-empty bin whose minimum lies more
// than the gap beyond the maximum of the previous non-empty bin.
__global__ void __launch_bounds__(1024) k_breakup_scan(const uint32_t* bin_base, const unsigned long long* bmin,
                                                      const unsigned long long* bmax, const double* start,
                                                      const double* gap, double* length, int32_t* broken) {
    __shared__ int last_ne[1024];
    __shared__ int found;
    __shared__ unsigned long long tip;
    const int s = blockIdx.x;
    const int b0 = (int)bin_base[s], b1 = (int)bin_base[s + 1];
    const int nt = (int)blockDim.x, t = (int)threadIdx.x;
    const int chunk = (b1 - b0 + nt - 1) / nt;
    const int i0 = b0 + t * chunk, i1 = min(i0 + chunk, b1);
    if (t == 0) {
        found = 0x7FFFFFFF;
        tip = 0ull;
    }
    // the last non-empty bin of this thread's run of bins
    int last = -1;
    unsigned long long hi = 0ull;
    for (int i = i0; i < i1; ++i) {
        const unsigned long long m = bmax[i];
        if (m != 0ull) {
            last = i;
            hi = m > hi ? m : hi;
        }
    }
    last_ne[t] = last;
    __syncthreads();
    if (hi) atomicMax(&tip, hi);
    // the last non-empty bin before this run: a maximum over the runs below
    int prev = -1;
    for (int k = 0; k < t; ++k) prev = last_ne[k] > prev ? last_ne[k] : prev;
    const double g = gap[s];
    for (int i = i0; i < i1; ++i) {
        if (bmax[i] == 0ull) continue;
        if (prev >= 0 && from_ordered(bmin[i]) - from_ordered(bmax[prev]) > g) {
            atomicMin(&found, prev);
            break;
        }
        prev = i;
    }
    __syncthreads();
    if (t == 0) {
        if (found != 0x7FFFFFFF) {
            length[s] = from_ordered(bmax[found]) - start[s];
            broken[s] = 1;
        } else {
            length[s] = tip ? from_ordered(tip) - start[s] : 0.0;
            broken[s] = 0;
        }
    }
}

void launch_breakup(int n, int n_sys, const uint32_t* tag, const double2* pos, double ax, double ay,
                    const double* start, unsigned long long* extent, hipStream_t st) {
    launch_fill_u64(extent, (size_t)n_sys, 0ull, st);
    k_breakup_extent<float><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, tag, pos, ax, ay, start, extent);
}

void launch_breakup_bins(int n, int n_sys, const uint32_t* tag, const double2* pos, double ax, double ay,
                         const double* start, const double* anchor, const double* half_gap, const double* gap,
                         const uint32_t* bin_base, uint32_t n_bins, unsigned long long* bmin, unsigned long long* bmax,
                         double* length, int32_t* broken, hipStream_t st) {
    launch_fill_u64(bmin, n_bins, ~0ull, st);
    launch_fill_u64(bmax, n_bins, 0ull, st);
    k_breakup_bins<float><<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, tag, pos, ax, ay, start, anchor, half_gap,
                                                                       bin_base, bmin, bmax);
    k_breakup_scan<<<(unsigned)n_sys, 1024, 0, st>>>(bin_base, bmin, bmax, start, gap, length, broken);
}

// Derived per-slot quantities for sph_read.
template <typename T>
__global__ void k_pressure(int n, const SysDev<T>* sys, const uint32_t* tag, const T* dens, T* out) {
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    uint32_t t = tag[a];
    out[a] = tait_pressure(sys[tag_sys(t)], dens[a]);
}

// A plain copy of known size: the reference point for HBM byte counters.
__global__ void k_copy_u32x4(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// ------------------------------------------------------------------ launchers

static inline unsigned nblk(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

void launch_fill_u32(uint32_t* p, size_t n, uint32_t v, hipStream_t st) {
    if (n) k_fill_u32<<<nblk((int64_t)n, 256), 256, 0, st>>>(p, n, v);
}
void launch_fill_u64(unsigned long long* p, size_t n, unsigned long long v, hipStream_t st) {
    if (n) k_fill_u64<<<nblk((int64_t)n, 256), 256, 0, st>>>(p, n, v);
}

int64_t scan_tiles(int64_t m) { return (m + SCAN_TILE - 1) / SCAN_TILE; }

// in[0..m) -> out[0..m] (in == out allowed unless clear_in); part holds
// scan_tiles(m) + 1 words. Up to 32 tiles go to the one-workgroup kernel.
static void launch_scan(uint32_t* in, uint32_t* out, int64_t m, bool clear_in, uint32_t* part, hipStream_t st,
                        KernelTimer* kt) {
    const int64_t nt = scan_tiles(m);
    kt->begin("scan", st);
    if (nt <= 32 && !clear_in) {
        k_scan_single<<<1, 1024, 0, st>>>(in, out, m);
    } else {
        k_scan_reduce<<<(unsigned)nt, SCAN_THREADS, 0, st>>>(in, m, part);
        k_scan_single<<<1, 1024, 0, st>>>(part, part, nt);
        k_scan_apply<<<(unsigned)nt, SCAN_THREADS, 0, st>>>(in, out, m, part, clear_in ? 1 : 0);
    }
    kt->end(st);
}

void copy_kernel(const void* src, void* dst, size_t bytes, hipStream_t st) {
    size_t n = bytes / 16;
    k_copy_u32x4<<<nblk((int64_t)n, 256), 256, 0, st>>>((const uint4*)src, (uint4*)dst, n);
}

template <typename T>
void launch_key(const LaunchCfg& L, const SortBufs& B, const SysDev<T>* sys, StateBuf<T> X, hipStream_t st,
                KernelTimer* kt) {
    kt->begin("sort_key", st);
    k_key<T><<<nblk(L.n, L.block_stream), L.block_stream, 0, st>>>(L.n, sys, X.pos, X.tag, B.key, B.slot, B.count,
                                                                    B.trash, B.blk);
    kt->end(st);
}

template <typename T>
void launch_sort(const LaunchCfg& L, const SortBufs& B, const SysDev<T>* sys, StateBuf<T> X, StateBuf<T> Y,
                 T* vol, bool keyed, hipStream_t st, KernelTimer* kt) {
    const int n = L.n;
    const int bs = L.block_stream;
    const uint32_t trash = B.trash;
    const unsigned nb = nblk(n, bs);
    // keyed: the corrector that produced X already wrote its keys, slots and
    // counts. Otherwise the per-cell counts are zero here: the cell scan of
    // the previous sort cleared them (and the first sort finds them cleared)
    if (!keyed) launch_key<T>(L, B, sys, X, st, kt);
    launch_scan(B.count, B.cstart, (int64_t)trash + 1, true, B.part, st, kt);
    launch_scan(B.blk, B.blk, (int64_t)nb, false, B.part2, st, kt);
    kt->begin("sort_scatter", st);
    k_scatter<<<nb, bs, 0, st>>>(n, B.key, B.slot, X.id, B.cstart, trash, B.cell_ids);
    kt->end(st);
    kt->begin("sort_permute", st);
    k_permute<T><<<nb, bs, 0, st>>>(n, sys, B.key, B.cstart, B.cell_ids, trash, B.blk, X, Y, B.cell, vol);
    kt->end(st);
    kt->begin("wave_table", st);
    k_wave_table<<<1, 1024, 0, st>>>(L.n_sys, B.sys_cell_base, B.cstart, B.sys_lo, B.sys_hi, B.chunk_base,
                                     B.surf_count);
    kt->end(st);
}

int64_t surface_chunks(int64_t n, int n_sys) { return (n + 63) / 64 + n_sys; }

int64_t surface_region(int64_t n, int n_sys) {
    const int64_t blocks = (surface_chunks(n, n_sys) + SURF_BLOCK - 1) / SURF_BLOCK;
    return (blocks + SURF_REGIONS - 1) / SURF_REGIONS * SURF_BLOCK * 64;
}

// The surface kernel's grid: enough waves for a list of 1/16 of the
// particles in one pass, at least 256 workgroups.
static unsigned surface_blocks(int64_t n) {
    const int64_t want = (n / 16 + 255) / 256;
    return (unsigned)(want < 256 ? 256 : (want > 4096 ? 4096 : want));
}

template <typename T>
void launch_eval(const LaunchCfg& L, const EvalView<T>& v, const WallView* W, hipStream_t st, KernelTimer* kt) {
    const int bs = L.block_sweep;
    const int64_t max_waves = ((int64_t)L.n + 63) / 64 + v.n_sys;
    const unsigned nb = nblk(max_waves, bs / 64);
    // the half step (v.skin_max set) follows each sweep with its RESCAN
    // kernel, which returns at once unless some system outran the skin mask
    const bool half = v.skin_max != nullptr;
    if (v.density_sum) {
        kt->begin("density", st);
        k_density<T><<<nb, bs, 0, st>>>(v);
        kt->end(st);
    }
    if (W) {   // repulsive-force walls: their force, from this evaluation's state
        kt->begin("wall_force", st);
        k_wall_force<T><<<nblk(L.n, 256), 256, 0, st>>>(v, *W);
        kt->end(st);
    }
    if (!v.smask) {
        kt->begin("colour_skin", st);
        k_colour_skin<T><<<nb, bs, 0, st>>>(v);
    } else {
        // the first evaluation of a step: the cell scan that writes the mask
        kt->begin("colour", st);
        k_colour<T><<<nb, bs, 0, st>>>(v);
    }
    kt->end(st);
    if (half) {
        kt->begin("rescan", st);
        k_colour_rescan<T><<<RESCAN_BLOCKS, 256, 0, st>>>(v);
        kt->end(st);
    }
    kt->begin("main", st);
    k_main<T><<<nb, bs, 0, st>>>(v);
    kt->end(st);
    if (half) {
        kt->begin("rescan", st);
        k_main_rescan<T><<<RESCAN_BLOCKS, 256, 0, st>>>(v);
        kt->end(st);
    }
    kt->begin("surface", st);
    const unsigned sb = surface_blocks(L.n);
    k_surface<T><<<sb + (half ? (unsigned)RESCAN_BLOCKS : 0u), 256, 0, st>>>(v, sb);
    kt->end(st);
}

template <typename T>
void launch_dt(int n_sys, const SysDev<T>* sys, const uint32_t* chunk_base, const double* dt_wave,
               unsigned long long* dtmin, double* dt, unsigned long long* skin_max, hipStream_t st, KernelTimer* kt) {
    kt->begin("dt", st);
    k_dt_finalize<T><<<(unsigned)n_sys, 1024, 0, st>>>(n_sys, sys, chunk_base, dt_wave, dtmin, dt, skin_max);
    kt->end(st);
}

template <typename T>
void launch_predict(const LaunchCfg& L, const IntegView<T>& v, hipStream_t st, KernelTimer* kt) {
    kt->begin("predict", st);
    k_predict<T><<<nblk(L.n, L.block_stream), L.block_stream, 0, st>>>(v);
    kt->end(st);
}

template <typename T>
void launch_correct(const LaunchCfg& L, const IntegView<T>& v, int n_sys, const double* dt, double* time,
                    hipStream_t st, KernelTimer* kt) {
    kt->begin("correct", st);
    k_correct<T><<<nblk(L.n, L.block_stream), L.block_stream, 0, st>>>(v);
    kt->end(st);
    kt->begin("time", st);
    k_advance_time<<<nblk(n_sys, 64), 64, 0, st>>>(n_sys, dt, time);
    kt->end(st);
}

// The first colour sweep alone: colour, neighbour record and the skin mask.
template <typename T>
void launch_colour_mask(const LaunchCfg& L, const EvalView<T>& v, hipStream_t st) {
    const int bs = L.block_sweep;
    const int64_t max_waves = ((int64_t)L.n + 63) / 64 + v.n_sys;
    k_colour<T><<<nblk(max_waves, bs / 64), bs, 0, st>>>(v);
}

template <typename T>
void launch_nbr_count(const LaunchCfg& L, const EvalView<T>& v, uint32_t* count, hipStream_t st) {
    k_nbr_count<T><<<nblk(L.n, 256), 256, 0, st>>>(v, count);
}

template <typename T>
void launch_nbr_fill(const EvalView<T>& v, int a0, int a1, const int64_t* start, int64_t base, uint32_t* out,
                     hipStream_t st) {
    if (a1 > a0) k_nbr_fill<T><<<nblk(a1 - a0, 256), 256, 0, st>>>(v, a0, a1, start, base, out);
}

template <typename T>
void launch_pressure(int n, const SysDev<T>* sys, const uint32_t* tag, const T* dens, T* out, hipStream_t st) {
    k_pressure<T><<<nblk(n, 256), 256, 0, st>>>(n, sys, tag, dens, out);
}

#define SPHJET_INSTANTIATE(T)                                                                               \
    template void launch_key<T>(const LaunchCfg&, const SortBufs&, const SysDev<T>*, StateBuf<T>,         \
                                hipStream_t, KernelTimer*);                                                \
    template void launch_sort<T>(const LaunchCfg&, const SortBufs&, const SysDev<T>*, StateBuf<T>,        \
                                 StateBuf<T>, T*, bool, hipStream_t, KernelTimer*);                        \
    template void launch_eval<T>(const LaunchCfg&, const EvalView<T>&, const WallView*, hipStream_t,      \
                                 KernelTimer*);                                                            \
    template void launch_dt<T>(int, const SysDev<T>*, const uint32_t*, const double*, unsigned long long*, \
                               double*, unsigned long long*, hipStream_t,                                  \
                               KernelTimer*);                                                              \
    template void launch_predict<T>(const LaunchCfg&, const IntegView<T>&, hipStream_t, KernelTimer*);     \
    template void launch_correct<T>(const LaunchCfg&, const IntegView<T>&, int, const double*, double*,    \
                                    hipStream_t, KernelTimer*);                                            \
    template void launch_colour_mask<T>(const LaunchCfg&, const EvalView<T>&, hipStream_t);               \
    template void launch_nbr_count<T>(const LaunchCfg&, const EvalView<T>&, uint32_t*, hipStream_t);       \
    template void launch_nbr_fill<T>(const EvalView<T>&, int, int, const int64_t*, int64_t, uint32_t*,    \
                                     hipStream_t);                                                         \
    template void launch_pressure<T>(int, const SysDev<T>*, const uint32_t*, const T*, T*, hipStream_t);

SPHJET_INSTANTIATE(float)
SPHJET_INSTANTIATE(double)

}  // namespace sphjet

// Learned curvature closure: stencil construction, a 64 -> 64 -> 64 -> 3 MLP
// (tanh hidden layers, linear output: n_x, n_y, kappa h) on BF16 MFMA with
// FP32 accumulation, its training (forward, backward, Adam), and the closure
// step that puts the network's curvature into the surface-tension term of
// eq. 24 with the plain estimate of eq. 23 as fallback.
//
// Matrix tiles use v_mfma_f32_16x16x16_bf16: for a 16x16 A (rows x k), a
// 16x16 B (k x cols) and the 16x16 FP32 result, lane l holds
//   A[l % 16][4 (l / 16) + i],  B[4 (l / 16) + i][l % 16],  D[4 (l / 16) + i][l % 16],  i = 0..3.
// Weights are kept in BF16 twice: transposed (out x in, row-major) so that the
// forward B fragments are 8 contiguous bytes per lane, and as stored (in x
// out, row-major) for the backward products with W^T. Every kernel here runs
// one wavefront per workgroup, so __syncthreads() is a wave barrier.
#include <algorithm>

#include "sph_internal.hpp"

namespace sphjet {

typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ bf4 pack4(float a, float b, float c, float d) {
    bf4 r;
    r.x = (short)f2bf(a);
    r.y = (short)f2bf(b);
    r.z = (short)f2bf(c);
    r.w = (short)f2bf(d);
    return r;
}
__device__ __forceinline__ bf4 load4(const uint16_t* p) { return *reinterpret_cast<const bf4*>(p); }
__device__ __forceinline__ f4 mfma(bf4 a, bf4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 zero4() { f4 z = {0.f, 0.f, 0.f, 0.f}; return z; }

// Sum over the 64 lanes that share l % 16 (a column of a D tile), all four
// entries: result valid in every lane.
__device__ __forceinline__ float colsum(f4 v) {
    float s = v.x + v.y + v.z + v.w;
    s += __shfl_xor(s, 16, 64);
    s += __shfl_xor(s, 32, 64);
    return s;
}

// ----------------------------------------------------------------- forward

// tanh x = 1 - 2 / (e^{2x} + 1) from the hardware exp2 and reciprocal. Its
// absolute error (about 1e-7) is far below the BF16 rounding the hidden
// activations get next; the limits give exactly +-1.
__device__ __forceinline__ float tanh_fast(float x) {
    const float e = __builtin_amdgcn_exp2f(x * 2.8853900817779268f);   // e^{2x} = 2^{2x / ln 2}
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

// The B fragments and biases this lane needs, read from the weights in memory
// (the training kernel, whose registers hold the gradient sums) ...
struct WMem {
    const MlpView& W;
    __device__ bf4 w1(int nb, int kb, int r, int g) const { return load4(W.wt1 + (16 * nb + r) * 64 + 16 * kb + 4 * g); }
    __device__ bf4 w2(int nb, int kb, int r, int g) const { return load4(W.wt2 + (16 * nb + r) * 64 + 16 * kb + 4 * g); }
    __device__ bf4 w3(int kb, int r, int g) const { return load4(W.wt3 + r * 64 + 16 * kb + 4 * g); }
    __device__ float b1(int nb, int r) const { return W.b1[16 * nb + r]; }
    __device__ float b2(int nb, int r) const { return W.b2[16 * nb + r]; }
    __device__ float b3(int r) const { return W.b3[r]; }
};

// ... or held in registers for every tile a wave processes (72 VGPRs of
// fragments, loaded once per wave).
struct WReg {
    bf4 f1[4][4], f2[4][4], f3[4];
    float c1[4], c2[4], c3;
    __device__ void load(const MlpView& W) {
        const int l = __lane_id(), r = l & 15, g = l >> 4;
        const WMem M{W};
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) {
                f1[nb][kb] = M.w1(nb, kb, r, g);
                f2[nb][kb] = M.w2(nb, kb, r, g);
            }
            c1[nb] = M.b1(nb, r);
            c2[nb] = M.b2(nb, r);
        }
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) f3[kb] = M.w3(kb, r, g);
        c3 = M.b3(r);
    }
    __device__ bf4 w1(int nb, int kb, int, int) const { return f1[nb][kb]; }
    __device__ bf4 w2(int nb, int kb, int, int) const { return f2[nb][kb]; }
    __device__ bf4 w3(int kb, int, int) const { return f3[kb]; }
    __device__ float b1(int nb, int) const { return c1[nb]; }
    __device__ float b2(int nb, int) const { return c2[nb]; }
    __device__ float b3(int) const { return c3; }
};

// One 16-row tile through the network. X: 16 x 64 BF16 in LDS (row-major).
// h1, h2: LDS scratch 16 x 64 BF16. Returns the layer outputs in D layout:
// H1[nb], H2[nb] (FP32, 4 column blocks) and Y (columns 0..2 valid).
template <typename WS>
__device__ __forceinline__ void mlp_tile_forward(const WS& W, const uint16_t* xs, uint16_t* h1s, uint16_t* h2s,
                                                 f4 H1[4], f4 H2[4], f4& Y) {
    const int l = __lane_id(), r = l & 15, g = l >> 4;
    bf4 xa[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) xa[kb] = load4(xs + r * 64 + 16 * kb + 4 * g);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        f4 acc = zero4();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma(xa[kb], W.w1(nb, kb, r, g), acc);
        const float bias = W.b1(nb, r);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float h = tanh_fast(acc[i] + bias);
            acc[i] = h;
            h1s[(4 * g + i) * 64 + 16 * nb + r] = f2bf(h);
        }
        H1[nb] = acc;
    }
    __syncthreads();
    bf4 ha[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) ha[kb] = load4(h1s + r * 64 + 16 * kb + 4 * g);
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
        f4 acc = zero4();
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) acc = mfma(ha[kb], W.w2(nb, kb, r, g), acc);
        const float bias = W.b2(nb, r);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            float h = tanh_fast(acc[i] + bias);
            acc[i] = h;
            h2s[(4 * g + i) * 64 + 16 * nb + r] = f2bf(h);
        }
        H2[nb] = acc;
    }
    __syncthreads();
    f4 acc = zero4();
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma(load4(h2s + r * 64 + 16 * kb + 4 * g), W.w3(kb, r, g), acc);
    const float bias = W.b3(r);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] += bias;
    Y = acc;
}

// Copy rows [row0, row0 + 16) of X (m x 64 BF16) into LDS, zero past m.
__device__ __forceinline__ void load_tile(const uint16_t* X, int64_t m, int64_t row0, uint16_t* xs) {
    const int l = __lane_id();
    // 16 rows x 64 = 1024 BF16 = 256 x 8 bytes: four 8-byte chunks per lane
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int chunk = c * 64 + l;
        int rr = chunk >> 4, cc = (chunk & 15) * 4;
        bf4 v = {0, 0, 0, 0};
        if (row0 + rr < m) v = load4(X + (row0 + rr) * 64 + cc);
        *reinterpret_cast<bf4*>(xs + rr * 64 + cc) = v;
    }
    __syncthreads();
}

// Y (m x 3, row stride ystride) = network(X) for every row; one wave walks
// the tiles.
__global__ void __launch_bounds__(64) k_mlp_forward(MlpView W, const uint16_t* X, int64_t m, float* Y,
                                                    int ystride) {
    __shared__ uint16_t xs[16 * 64], h1s[16 * 64], h2s[16 * 64];
    const int l = __lane_id(), r = l & 15, g = l >> 4;
    const int64_t ntiles = (m + 15) / 16;
    WReg F;
    F.load(W);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        load_tile(X, m, t * 16, xs);
        f4 H1[4], H2[4], y;
        mlp_tile_forward(F, xs, h1s, h2s, H1, H2, y);
        if (r < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int64_t row = t * 16 + 4 * g + i;
                if (row < m) Y[row * ystride + r] = y[i];
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- training

// Forward and backward of the mean squared error over m rows (targets T, m x 3);
// each wave accumulates the weight and bias gradients of its tiles in
// registers and writes them, in the flat parameter order (W1 in x out, b1, W2,
// b2, W3 in x 3, b3), to partial[wave]; loss_part[wave] gets its sum of
// squared errors.
__global__ void __launch_bounds__(64) k_mlp_grad(MlpView W, const uint16_t* X, const float* T, int64_t m,
                                                 int tiles_per_wave, float* partial, float* loss_part) {
    __shared__ uint16_t xs[16 * 64], h1s[16 * 64], h2s[16 * 64], ts[16 * 64];
    const int l = __lane_id(), r = l & 15, g = l >> 4;
    const float gscale = 2.0f / (float)(m * 3);
    f4 dW1[4][4], dW2[4][4], dW3[4];
    float db1[4] = {0, 0, 0, 0}, db2[4] = {0, 0, 0, 0}, db3 = 0.f, lsum = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        dW3[a] = zero4();
#pragma unroll
        for (int b = 0; b < 4; ++b) { dW1[a][b] = zero4(); dW2[a][b] = zero4(); }
    }
    const int64_t ntiles = (m + 15) / 16;
    for (int k = 0; k < tiles_per_wave; ++k) {
        const int64_t t = (int64_t)blockIdx.x * tiles_per_wave + k;
        if (t >= ntiles) break;
        const int64_t row0 = t * 16;
        load_tile(X, m, row0, xs);
        f4 H1[4], H2[4], y;
        mlp_tile_forward(WMem{W}, xs, h1s, h2s, H1, H2, y);
        // output error: dY = 2 (Y - T) / (3 m) on valid rows and columns
        f4 dY;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            int64_t row = row0 + 4 * g + i;
            float d = 0.f;
            if (row < m && r < 3) {
                d = y[i] - T[row * 3 + r];
                lsum += d * d;
            }
            dY[i] = d * gscale;
        }
        // dW3 = H2^T dY, db3 = colsum(dY)
        bf4 dyb = pack4(dY[0], dY[1], dY[2], dY[3]);
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) dW3[mb] = mfma(pack4(H2[mb][0], H2[mb][1], H2[mb][2], H2[mb][3]), dyb, dW3[mb]);
        db3 += colsum(dY);
        // dH2 = dY W3^T: dY to A layout through LDS (16 x 16 in the first columns of ts)
#pragma unroll
        for (int i = 0; i < 4; ++i) ts[(4 * g + i) * 64 + r] = f2bf(dY[i]);
        __syncthreads();
        bf4 dya = load4(ts + r * 64 + 4 * g);
        f4 dZ2[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            f4 acc = mfma(dya, load4(W.w3 + (16 * nb + r) * 16 + 4 * g), zero4());
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] *= 1.f - H2[nb][i] * H2[nb][i];
            dZ2[nb] = acc;
            db2[nb] += colsum(acc);
        }
        __syncthreads();
        // dW2 = H1^T dZ2
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            bf4 a = pack4(H1[mb][0], H1[mb][1], H1[mb][2], H1[mb][3]);
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                dW2[mb][nb] = mfma(a, pack4(dZ2[nb][0], dZ2[nb][1], dZ2[nb][2], dZ2[nb][3]), dW2[mb][nb]);
        }
        // dH1 = dZ2 W2^T: dZ2 to A layout through LDS
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) ts[(4 * g + i) * 64 + 16 * nb + r] = f2bf(dZ2[nb][i]);
        __syncthreads();
        bf4 dza[4];
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) dza[kb] = load4(ts + r * 64 + 16 * kb + 4 * g);
        f4 dZ1[4];
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            f4 acc = zero4();
#pragma unroll
            for (int kb = 0; kb < 4; ++kb) acc = mfma(dza[kb], load4(W.w2 + (16 * nb + r) * 64 + 16 * kb + 4 * g), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) acc[i] *= 1.f - H1[nb][i] * H1[nb][i];
            dZ1[nb] = acc;
            db1[nb] += colsum(acc);
        }
        // dW1 = X^T dZ1: the A fragment of X^T is X in D layout, read from LDS
#pragma unroll
        for (int mb = 0; mb < 4; ++mb) {
            bf4 a;
            a.x = (short)xs[(4 * g + 0) * 64 + 16 * mb + r];
            a.y = (short)xs[(4 * g + 1) * 64 + 16 * mb + r];
            a.z = (short)xs[(4 * g + 2) * 64 + 16 * mb + r];
            a.w = (short)xs[(4 * g + 3) * 64 + 16 * mb + r];
#pragma unroll
            for (int nb = 0; nb < 4; ++nb)
                dW1[mb][nb] = mfma(a, pack4(dZ1[nb][0], dZ1[nb][1], dZ1[nb][2], dZ1[nb][3]), dW1[mb][nb]);
        }
        __syncthreads();
    }
    // write this wave's partial sums in the flat parameter order
    float* P = partial + (size_t)blockIdx.x * MLP_NPARAMS;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int nb = 0; nb < 4; ++nb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                int in = 16 * mb + 4 * g + i, out = 16 * nb + r;
                P[MLP_OFF_W1 + in * 64 + out] = dW1[mb][nb][i];
                P[MLP_OFF_W2 + in * 64 + out] = dW2[mb][nb][i];
            }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (r < 3) P[MLP_OFF_W3 + (16 * mb + 4 * g + i) * 3 + r] = dW3[mb][i];
    if (g == 0) {
#pragma unroll
        for (int nb = 0; nb < 4; ++nb) {
            P[MLP_OFF_B1 + 16 * nb + r] = db1[nb];
            P[MLP_OFF_B2 + 16 * nb + r] = db2[nb];
        }
        if (r < 3) P[MLP_OFF_B3 + r] = db3;
    }
    // the wave's sum of squared errors
    float s = lsum;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if (l == 0) loss_part[blockIdx.x] = s;
}

// grad[p] = sum over waves of partial[w][p], in wave order (deterministic).
__global__ void k_mlp_reduce(const float* partial, int nwaves, float* grad, const float* loss_part, float* loss,
                             float loss_scale) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < MLP_NPARAMS) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += partial[(size_t)w * MLP_NPARAMS + p];
        grad[p] = s;
    }
    if (p == 0 && loss) {
        float s = 0.f;
        for (int w = 0; w < nwaves; ++w) s += loss_part[w];
        *loss = s * loss_scale;
    }
}

// Write the BF16 copies of parameter p (FP32 master value w) in both layouts.
__device__ __forceinline__ void write_bf16(MlpBufs B, int p, float w) {
    uint16_t b = f2bf(w);
    if (p < MLP_OFF_B1) {
        int in = p / 64, out = p % 64;
        B.wt1[out * 64 + in] = b;
    } else if (p < MLP_OFF_W2) {
        B.b1[p - MLP_OFF_B1] = w;
    } else if (p < MLP_OFF_B2) {
        int q = p - MLP_OFF_W2, in = q / 64, out = q % 64;
        B.wt2[out * 64 + in] = b;
        B.w2[in * 64 + out] = b;
    } else if (p < MLP_OFF_W3) {
        B.b2[p - MLP_OFF_B2] = w;
    } else if (p < MLP_OFF_B3) {
        int q = p - MLP_OFF_W3, in = q / 3, out = q % 3;
        B.wt3[out * 64 + in] = b;
        B.w3[in * 16 + out] = b;
    } else {
        B.b3[p - MLP_OFF_B3] = w;
    }
}

// Load FP32 parameters and write their BF16 working copies.
__global__ void k_mlp_set(MlpBufs B, const float* params) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAMS) return;
    float w = params[p];
    B.master[p] = w;
    write_bf16(B, p, w);
}

// Adam on the FP32 masters (step t >= 1), then the BF16 copies.
__global__ void k_mlp_adam(MlpBufs B, const float* grad, float lr, float b1, float b2, float eps, float c1,
                           float c2) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= MLP_NPARAMS) return;
    float gr = grad[p];
    float m = b1 * B.adam_m[p] + (1.f - b1) * gr;
    float v = b2 * B.adam_v[p] + (1.f - b2) * gr * gr;
    B.adam_m[p] = m;
    B.adam_v[p] = v;
    float w = B.master[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
    B.master[p] = w;
    write_bf16(B, p, w);
}

// ----------------------------------------------------------------- closure

// Position of the i-th set bit of the 32-bit word m (0-based); m must have
// more than i set bits.
__device__ __forceinline__ int select_bit(uint32_t m, int i) {
    int pos = 0;
#pragma unroll
    for (int w = 16; w >= 1; w >>= 1) {
        const uint32_t low = (1u << w) - 1u;
        const int c = __popc(m & low);
        if (i >= c) {
            i -= c;
            m >>= w;
            pos += w;
        } else {
            m &= low;
        }
    }
    return pos;
}

// Candidates of a listed slot: the set bits of its mask words, or, when the
// mask overflowed, every slot of its block up to the 128th. The distance test
// is redone for each candidate (a skin mask also holds pairs out to R s).
__device__ __forceinline__ int stencil_candidates(const RowMask& M) {
    if (M.w[4] & MASK_OVERFLOW) return 128;
    return __popc(M.w[0]) + __popc(M.w[1]) + __popc(M.w[2]) + __popc(M.w[3]) + __popc(M.w[4]);
}

__device__ __forceinline__ RowMask closure_mask(const uint4* nmask, const uint32_t* nmask4, uint32_t a) {
    const uint4 w = nmask[a];
    RowMask M;
    M.w[0] = w.x;
    M.w[1] = w.y;
    M.w[2] = w.z;
    M.w[3] = w.w;
    M.w[4] = nmask4[a];
    return M;
}

// One listed slot's stencil, built by a group of `width` lanes (16, 32 or 64)
// of the wave, each lane taking candidates j and j + width, so a group takes
// at most 2 width of them; `a` is the slot, `M` its mask words, `j` the lane's
// index in the group and `lds` the group's 2 width LDS slots. Every lane of the
// wave calls this the same number of times (barriers); inactive groups pass
// active = false.
template <typename T>
__device__ __forceinline__ void build_stencil(const EvalView<T>& v, const ClosureView& C, uint32_t row, bool active,
                                              uint32_t a, const RowMask& M, int base, int width, int j, float* sx,
                                              float* sy, float* sd, float* sa, uint32_t* sid, uint32_t* skeep) {
    const int l = __lane_id();
    const int total = active ? stencil_candidates(M) : 0;
    const bool overflow = (M.w[4] & MASK_OVERFLOW) != 0;
    float ix[2] = {0.f, 0.f}, iy[2] = {0.f, 0.f}, id2[2] = {0.f, 0.f}, ian[2] = {0.f, 0.f};
    uint32_t iid[2] = {0u, 0u};
    bool val[2] = {false, false};
    if (active) {
        const SysDev<T>& S = v.sys[tag_sys(v.tag[a])];
        const double2 pa = v.pos[a];
        const uint32_t ny = (uint32_t)S.ny;
        const uint32_t local = v.cell[a] - S.cell_base;
        const int cx = (int)(local / ny), cy = (int)(local - (uint32_t)cx * ny);
        const int R = S.reach;
        const int ylo = cy - R < 0 ? 0 : cy - R, yhi = cy + R > S.ny - 1 ? S.ny - 1 : cy + R;
        const int xlo = cx - R < 0 ? 0 : cx - R, xhi = cx + R > S.nx - 1 ? S.nx - 1 : cx + R;
        const float ih = 1.0f / (float)S.h;
        // e1: unit colour gradient (eq. 18, into the liquid); e2: e1 turned by +90 degrees
        const V2<T> na = v.nrm[a];
        const float nfx = (float)na.x, nfy = (float)na.y;
        const float inv_n = 1.0f / sqrtf(nfx * nfx + nfy * nfy);
        const float e1x = nfx * inv_n, e1y = nfy * inv_n;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int idx = j + width * it;
            if (idx >= total) continue;
            // the idx-th candidate: the idx-th set bit over the rows' words (its
            // row found from the words' bit counts, then one cell-start load),
            // or, after an overflow, the idx-th slot of the block
            uint32_t b = 0xFFFFFFFFu;
            if (!overflow) {
                uint32_t ord0 = 0, wsel = 0, k = 0;
                int rsel = -1;
#pragma unroll
                for (int r = 0; r < 5; ++r) {
                    const uint32_t cnt = (uint32_t)__popc(M.w[r]);
                    const bool here = rsel < 0 && (uint32_t)idx < ord0 + cnt;
                    rsel = here ? r : rsel;
                    wsel = here ? M.w[r] : wsel;
                    k = here ? (uint32_t)idx - ord0 : k;
                    ord0 += cnt;
                }
                // rows past the grid edge have no bits, so rsel <= xhi - xlo
                if (rsel >= 0)
                    b = v.cstart[S.cell_base + (uint32_t)(xlo + rsel) * ny + ylo] + (uint32_t)select_bit(wsel, (int)k);
            } else {
                uint32_t ord0 = 0;
                for (int X = xlo; X <= xhi; ++X) {
                    const uint32_t rowc = S.cell_base + (uint32_t)X * ny;
                    const uint32_t b0 = v.cstart[rowc + ylo];
                    const uint32_t cnt = v.cstart[rowc + yhi + 1] - b0;
                    if ((uint32_t)idx < ord0 + cnt) {
                        b = b0 + ((uint32_t)idx - ord0);
                        break;
                    }
                    ord0 += cnt;
                }
            }
            if (b == 0xFFFFFFFFu || b == a) continue;
            // b is a slot of the block: its position, tag and id are loaded together
            const double2 pb = v.pos[b];
            const uint32_t tb = v.tag[b], idb = v.id[b];
            double ex, ey;
            const double r2 = pair_r2(pa, pb, ex, ey);
            // an overflowed mask lists every slot of the block, and the
            // half step's skin mask pairs out to R s: the exact predicate
            if (!(r2 < S.R2)) continue;
            if (tag_type(tb) != T_FLUID) continue;
            // relative position of b as seen from a, in units of h, then in the frame (e1, e2)
            const float x = -(float)ex * ih, y = -(float)ey * ih;
            const float xl = x * e1x + y * e1y, yl = y * e1x - x * e1y;
            float ang = atan2f(yl, xl);
            if (ang == -3.14159265358979323846f) ang = 3.14159265358979323846f;
            val[it] = true;
            ix[it] = xl;
            iy[it] = yl;
            id2[it] = x * x + y * y;
            ian[it] = ang;
            iid[it] = idb;
        }
    }
    // compact the group's valid items into its LDS slots [0, k)
    const unsigned long long gmask = width == 64 ? ~0ull : (((1ull << width) - 1ull) << base);
    const unsigned long long g0 = __ballot(val[0]) & gmask, g1 = __ballot(val[1]) & gmask;
    const int k0 = __popcll(g0), k = k0 + __popcll(g1);
    const unsigned long long below = (1ull << l) - 1ull;
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        if (val[it]) {
            const int p = it == 0 ? __popcll(g0 & below) : k0 + __popcll(g1 & below);
            sx[p] = ix[it];
            sy[p] = iy[it];
            sd[p] = id2[it];
            sa[p] = ian[it];
            sid[p] = iid[it];
        }
    }
    __syncthreads();
    // the 32 nearest (ties by id) stay
    bool keep[2] = {false, false};
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const int q0 = j + width * it;
        if (q0 < k) {
            int drank = 0;
            if (k > 32) {
                const float d = sd[q0];
                const uint32_t id = sid[q0];
                for (int q = 0; q < k; ++q) {
                    const float od = sd[q];
                    drank += (od < d || (od == d && sid[q] < id)) ? 1 : 0;
                }
            }
            keep[it] = drank < 32;
            skeep[q0] = keep[it] ? 1u : 0u;
        }
    }
    __syncthreads();
    // angle rank among the kept (ties: nearer, then lower id); write the row
    if (active) {
        uint16_t* out = C.stencil + (size_t)row * 64;
        const int nkept = k < 32 ? k : 32;
        for (int e = j; e < 64; e += width)
            if (e >= 2 * nkept) out[e] = 0;
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            const int q0 = j + width * it;
            if (q0 < k && keep[it]) {
                const float an = sa[q0], d = sd[q0];
                const uint32_t id = sid[q0];
                int arank = 0;
                for (int q = 0; q < k; ++q) {
                    const float oa = sa[q], od = sd[q];
                    const bool before = oa < an || (oa == an && (od < d || (od == d && sid[q] < id)));
                    arank += (skeep[q] != 0u && before) ? 1 : 0;
                }
                out[2 * arank] = f2bf(sx[q0]);
                out[2 * arank + 1] = f2bf(sy[q0]);
            }
        }
    }
    __syncthreads();  // the LDS slots are reused by the next call
}

// Stencil of each listed surface particle: the relative positions
// (r_b - r_a)/h of its fluid neighbours, the 32 nearest kept (ties by particle
// id), expressed in the frame e1 = n_a/|n_a| (eq. 18), e2 = e1 turned by +90
// degrees, ordered by their angle in that frame in (-pi, pi] (ties: nearer,
// then lower id; the cut at angle pi faces away from the liquid), zero-padded;
// written as 64 BF16 values per row. On a long list a wave takes four listed
// particles, one per 16 lanes, when each has at most 32 candidates (the usual
// case on a free surface); otherwise, and on a short list, it takes them two
// at a time, one per half (at most 64 candidates each), or one at a time with
// all 64 lanes. The kernel waits on chains of dependent loads: four chains per
// wave and eight waves per SIMD (at most 64 VGPRs, no spills) keep more of
// them in flight.
template <typename T>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8))) k_stencil(EvalView<T> v, ClosureView C) {
    __shared__ float sx[128], sy[128], sd[128], sa[128];
    __shared__ uint32_t sid[128], skeep[128];
    const int l = __lane_id();
    const uint32_t count = *C.count;
    // four rows per wave only when two per wave would already more than fill
    // the chip's wave slots; a short list keeps more waves at two rows each
    const uint32_t per = count > C.quad_min ? 4u : 2u;
    for (uint32_t q = blockIdx.x; per * q < count; q += gridDim.x) {
        const uint32_t end = per * q + per < count ? per * q + per : count;
        // rows r .. r + 64/width - 1, one per group of `width` lanes, each lane
        // taking candidates j and j + width: a group of 16 or 32 lanes is used
        // only when every one of its rows has at most 2 width candidates (a
        // wave-uniform test, so no lane reaches a barrier alone)
        uint32_t r = per * q;
        int width = per == 4u ? 16 : 32;
        while (r < end) {
            const int g = l / width;
            const uint32_t row = r + (uint32_t)g;
            const bool active = row < end;
            uint32_t a = 0;
            RowMask M = {{0u, 0u, 0u, 0u, 0u}};
            if (active) {
                a = C.list[row];
                M = closure_mask(v.nmask, v.nmask4, a);
            }
            if (width < 64 && __ballot(active && stencil_candidates(M) > 2 * width) != 0ull) {
                width *= 2;
                continue;
            }
            const int o = 2 * width * g;
            build_stencil<T>(v, C, row, active, a, M, width * g, width, l - width * g, sx + o, sy + o, sd + o,
                             sa + o, sid + o, skeep + o);
            r += (uint32_t)(64 / width);
            // after the first row of a pair built alone, its second alone too
            width = width == 64 && ((r & 1u) != 0u) ? 64 : 32;
        }
    }
}

// What the closure step of one listed particle reads besides the network's
// output; loaded before the network runs so the loads overlap its products.
template <typename T>
struct ApplyIn {
    uint32_t a;
    int sys;
    T h, tol, sigma, k_plain, rho;
    V2<T> n_a, acc;
    bool overflow;
};

template <typename T>
__device__ __forceinline__ ApplyIn<T> closure_apply_load(const EvalView<T>& v, uint32_t a) {
    ApplyIn<T> in;
    in.a = a;
    in.sys = (int)tag_sys(v.tag[a]);
    const SysDev<T>& S = v.sys[in.sys];
    in.h = S.h;
    in.tol = S.closure_tol;
    in.sigma = S.sigma;
    in.k_plain = v.kappa_plain[a];
    in.rho = v.eos[a].z;
    in.n_a = v.nrm[a];
    in.acc = v.acc[a];
    // the plain estimate is used where the stencil may be incomplete: the mask
    // overflowed, it holds more candidates than a stencil group takes (128), or
    // the half step of this system outran the skin mask the stencil walks
    const RowMask M = closure_mask(v.nmask, v.nmask4, a);
    in.overflow = (M.w[4] & MASK_OVERFLOW) != 0u || stencil_candidates(M) > 128 ||
                  (v.skin_max && v.skin_max[in.sys] != 0ull);
    return in;
}

// Surface-tension acceleration of one listed particle from the network's
// output y = (n_1, n_2, kappa h) (normal in the frame of n_a), or from the plain
// estimate where the network's curvature deviates from it by more than the
// tolerance (eq. 24); completes the total acceleration (eq. 25) and returns
// its eq. 30 limit.
template <typename T>
__device__ __forceinline__ double closure_apply_row(const EvalView<T>& v, const ClosureView& C,
                                                    const ApplyIn<T>& in, float y0, float y1, float y2) {
    const T k_mlp = (T)y2 / in.h;
    const T mag = sqrt_(in.n_a.x * in.n_a.x + in.n_a.y * in.n_a.y);
    // network normal from the frame (e1, e2) of n_a back to x, y
    const T e1x = in.n_a.x / mag, e1y = in.n_a.y / mag;
    T nx = (T)y0 * e1x - (T)y1 * e1y, ny = (T)y0 * e1y + (T)y1 * e1x;
    const T nm = sqrt_(nx * nx + ny * ny);
    const bool fb = fabs(k_mlp - in.k_plain) > in.tol * fabs(in.k_plain) || !(nm > T(0)) || in.overflow;
    T kappa;
    if (fb) {
        kappa = in.k_plain;
        nx = e1x;
        ny = e1y;
    } else {
        kappa = k_mlp;
        nx /= nm;
        ny /= nm;
    }
    const T f = -in.sigma / in.rho * kappa * mag;
    V2<T> acc = in.acc;
    acc.x += f * nx;
    acc.y += f * ny;
    v.acc[in.a] = acc;
    v.kappa[in.a] = kappa;
    C.fallback[in.a] = fb ? 1u : 0u;
    const T am = sqrt_(acc.x * acc.x + acc.y * acc.y);
    return am > T(0) ? sqrt((double)in.h / (double)am) : __builtin_inf();
}

// The network on the listed stencils, 16 rows per wave and tile, followed by
// the closure step of each row (one wavefront per workgroup).
template <typename T>
__global__ void __launch_bounds__(64) k_closure_net(EvalView<T> v, ClosureView C, MlpView W) {
    __shared__ uint16_t xs[16 * 64], h1s[16 * 64], h2s[16 * 64];
    __shared__ float ys[16 * 4];
    const int l = __lane_id(), r = l & 15, g = l >> 4;
    const int64_t m = (int64_t)*C.count;
    const int64_t ntiles = (m + 15) / 16;
    WReg F;
    F.load(W);
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int64_t row = t * 16 + l;
        const bool valid = l < 16 && row < m;
        ApplyIn<T> in{};
        if (valid) in = closure_apply_load<T>(v, C.list[row]);
        load_tile(C.stencil, m, t * 16, xs);
        f4 H1[4], H2[4], y;
        mlp_tile_forward(F, xs, h1s, h2s, H1, H2, y);
        if (r < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t rr = t * 16 + 4 * g + i;
                ys[(4 * g + i) * 4 + r] = y[i];
                if (rr < m) C.out[rr * 4 + r] = y[i];
            }
        }
        __syncthreads();
        double dtf = __builtin_inf();
        if (valid) dtf = closure_apply_row<T>(v, C, in, ys[l * 4], ys[l * 4 + 1], ys[l * 4 + 2]);
        if (v.do_dt) atomic_min_per_system(v.dtmin + 1, 2, in.sys, dtf, valid);
        __syncthreads();
    }
}

// ----------------------------------------------------------------- launchers

void launch_mlp_forward(const MlpView& W, const uint16_t* X, int64_t m, float* Y, int ystride, hipStream_t st) {
    int64_t ntiles = (m + 15) / 16;
    // every wave loads the weights once and walks several tiles
    unsigned grid = (unsigned)(ntiles < 2048 ? (ntiles > 0 ? ntiles : 1) : 2048);
    k_mlp_forward<<<grid, 64, 0, st>>>(W, X, m, Y, ystride);
}

// Waves of the gradient kernel for m rows: one per 16-row tile, at most
// MLP_GRAD_WAVES (each then takes a contiguous run of tiles), so the partial
// sums stay within MLP_GRAD_WAVES x MLP_NPARAMS floats.
int mlp_grad_waves(int64_t m) {
    const int64_t ntiles = (m + 15) / 16;
    return (int)std::max<int64_t>(1, std::min<int64_t>(ntiles, MLP_GRAD_WAVES));
}

void launch_mlp_grad(const MlpView& W, const uint16_t* X, const float* T, int64_t m, float* partial,
                     float* loss_part, float* grad, float* loss, hipStream_t st) {
    const int nw = mlp_grad_waves(m);
    const int64_t ntiles = (m + 15) / 16;
    const int tiles_per_wave = (int)((ntiles + nw - 1) / nw);
    k_mlp_grad<<<nw, 64, 0, st>>>(W, X, T, m, tiles_per_wave, partial, loss_part);
    k_mlp_reduce<<<(MLP_NPARAMS + 255) / 256, 256, 0, st>>>(partial, nw, grad, loss_part, loss,
                                                             1.0f / (float)(m * 3));
}

void launch_mlp_set(const MlpBufs& B, const float* params, hipStream_t st) {
    k_mlp_set<<<(MLP_NPARAMS + 255) / 256, 256, 0, st>>>(B, params);
}

void launch_mlp_adam(const MlpBufs& B, const float* grad, float lr, int t, hipStream_t st) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    k_mlp_adam<<<(MLP_NPARAMS + 255) / 256, 256, 0, st>>>(B, grad, lr, b1, b2, eps, c1, c2);
}

template <typename T>
void launch_closure(const EvalView<T>& v, const ClosureView& C, const MlpView& W, int64_t capacity, hipStream_t st,
                    KernelTimer* kt) {
    kt->begin("closure_stencil", st);
    // grids sized for the listed particles a system of this size can have
    // (a free surface lists a few percent), at least one wave per SIMD
    const unsigned sgrid = (unsigned)std::min<int64_t>(65536, std::max<int64_t>(1024, capacity / 64));
    k_stencil<T><<<sgrid, 64, 0, st>>>(v, C);
    kt->end(st);
    kt->begin("closure_net", st);
    // the network's waves load the weights once and walk several tiles each;
    // at most 3072 of them, one per wave slot of the chip at this kernel's three
    // waves per SIMD
    const unsigned ngrid = (unsigned)std::min<int64_t>(3072, std::max<int64_t>(256, capacity / 2048));
    k_closure_net<T><<<ngrid, 64, 0, st>>>(v, C, W);
    kt->end(st);
}

template void launch_closure<float>(const EvalView<float>&, const ClosureView&, const MlpView&, int64_t,
                                    hipStream_t, KernelTimer*);
template void launch_closure<double>(const EvalView<double>&, const ClosureView&, const MlpView&, int64_t,
                                     hipStream_t, KernelTimer*);

}  // namespace sphjet

// Learned importance proposal for hyperwedge sampling: per-wedge features,
// a 16 -> 64 -> 64 -> 1 ReLU network (float32), its forward and backward
// kernels and Adam.  The network regresses log(1 + closure count) of a
// hyperwedge; the sampler draws hyperwedges in proportion to the predicted
// count, mixed with a uniform floor.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "philox.hpp"

struct htri_model {
    htri::Allocator al;
    hipStream_t stream = nullptr;
    htri::DBuf<float> params;   // HTRI_MODEL_NUM_PARAMS
    htri::DBuf<float> adam_m, adam_v;
    int64_t adam_t = 0;
    std::string err;
};

namespace htri {

constexpr int kIn = 16, kH = 64;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * kIn, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH, kNumParams = kOffB3 + 1;
static_assert(kNumParams == HTRI_MODEL_NUM_PARAMS, "parameter layout");

namespace {

constexpr int kMaskWordsMax = 4;
__host__ __device__ __forceinline__ int mask_words(int size) {
    return size <= 32 * kMaskWordsMax ? (size + 31) / 32 : 0;
}

struct FeatArgs {
    const int64_t *fptr;
    const uint32_t *fadj;
    const int64_t *mptr;
    const uint32_t *fmask;
    const int32_t *esize;
    const int64_t *eptr;
    const int32_t *emem;
    const int64_t *vptr;
    const uint32_t *indeg;
    int64_t m;
    int wbits;
};

__device__ __forceinline__ int64_t owner_of_f(const int64_t *fptr, int64_t m, int64_t e) {
    int64_t lo = 0, hi = m;
    while (hi - lo > 1) {
        int64_t mid = (lo + hi) >> 1;
        if (fptr[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

// 16 features of hyperwedge e (owner r known)
__device__ void wedge_features(const FeatArgs &A, int64_t r, int64_t e, float *f) {
    const uint32_t ent = A.fadj[e];
    const uint32_t j = ent >> A.wbits;
    const int om = (int)(ent & ((1u << A.wbits) - 1));
    const int si = A.esize[r], sj = A.esize[j];
    const int64_t dr = A.fptr[r + 1] - A.fptr[r], dj = A.fptr[j + 1] - A.fptr[j];
    const int64_t pos = e - A.fptr[r];
    const int64_t after = dr - pos - 1;
    const int mn = si < sj ? si : sj, mx = si > sj ? si : sj;
    // degrees |E_v| over the shared vertices
    float dmax = 0.f, dmin = 1e30f, dsum = 0.f;
    int cnt = 0;
    const int W = mask_words(si);
    if (W > 0) {
        const int64_t mb = A.mptr[r] + pos * W;
        for (int w = 0; w < W; w++) {
            uint32_t bits = A.fmask[mb + w];
            while (bits) {
                int b = __ffs(bits) - 1;
                bits &= bits - 1;
                int32_t v = A.emem[A.eptr[r] + w * 32 + b];
                float dv = (float)(A.vptr[v + 1] - A.vptr[v]);
                dmax = fmaxf(dmax, dv);
                dmin = fminf(dmin, dv);
                dsum += dv;
                cnt++;
            }
        }
    } else {
        int64_t a = A.eptr[r], ae = A.eptr[r + 1], b = A.eptr[j], be = A.eptr[j + 1];
        while (a < ae && b < be) {
            int32_t x = A.emem[a], y = A.emem[b];
            if (x < y) a++;
            else if (y < x) b++;
            else {
                float dv = (float)(A.vptr[x + 1] - A.vptr[x]);
                dmax = fmaxf(dmax, dv);
                dmin = fminf(dmin, dv);
                dsum += dv;
                cnt++;
                a++;
                b++;
            }
        }
    }
    if (cnt == 0) dmin = 0.f;
    f[0] = log1pf((float)si);
    f[1] = log1pf((float)sj);
    f[2] = log1pf((float)om);
    f[3] = (om == mn) ? 1.f : 0.f;
    f[4] = log1pf((float)dr);
    f[5] = log1pf((float)dj);
    f[6] = log1pf((float)after);
    f[7] = log1pf((float)(after < dj ? after : dj));
    f[8] = log1pf((float)(dr + A.indeg[r]));
    f[9] = log1pf((float)(dj + A.indeg[j]));
    f[10] = (float)om / (float)mn;
    f[11] = (float)om / (float)mx;
    f[12] = log1pf(dmax);
    f[13] = log1pf(dmin);
    f[14] = log1pf(cnt ? dsum / (float)cnt : 0.f);
    f[15] = 1.f;
}

__global__ void k_features_all(FeatArgs A, int64_t nw, float *out) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < A.m;
         r += (int64_t)gridDim.x * blockDim.x) {
        for (int64_t e = A.fptr[r]; e < A.fptr[r + 1]; e++) {
            float f[kIn];
            wedge_features(A, r, e, f);
            for (int c = 0; c < kIn; c++) out[e * kIn + c] = f[c];
        }
    }
}

// network forward for one row, weights in LDS
__device__ __forceinline__ float mlp_forward_row(const float *P, const float *x) {
    float h1[kH];
#pragma unroll
    for (int o = 0; o < kH; o++) {
        float z = P[kOffB1 + o];
#pragma unroll
        for (int c = 0; c < kIn; c++) z = fmaf(P[kOffW1 + o * kIn + c], x[c], z);
        h1[o] = fmaxf(z, 0.f);
    }
    float out = P[kOffB3];
    for (int o = 0; o < kH; o++) {
        float z = P[kOffB2 + o];
#pragma unroll
        for (int i = 0; i < kH; i++) z = fmaf(P[kOffW2 + o * kH + i], h1[i], z);
        out = fmaf(P[kOffW3 + o], fmaxf(z, 0.f), out);
    }
    return out;
}

__global__ __launch_bounds__(256) void k_forward(const float *params, const float *x, int64_t n, float *out) {
    __shared__ float P[kNumParams];
    for (int t = threadIdx.x; t < kNumParams; t += blockDim.x) P[t] = params[t];
    __syncthreads();
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        float xr[kIn];
#pragma unroll
        for (int c = 0; c < kIn; c++) xr[c] = x[r * kIn + c];
        out[r] = mlp_forward_row(P, xr);
    }
}

// features + forward fused over a list of wedges: predicted closure count
// expm1(max(s, 0)) (s clamped) per wedge
// five waves per SIMD: the scores wait on the features' dependent gathers, and
// the row's work (a call, so that the two loops share it) fits 96 VGPRs
__global__ __launch_bounds__(256, 5) void k_score(FeatArgs A, const float *params, const int64_t *wedges, int64_t n,
                                               double *score) {
    __shared__ float P[kNumParams];
    __shared__ int64_t s_own[2];
    for (int t = threadIdx.x; t < kNumParams; t += blockDim.x) P[t] = params[t];
    __syncthreads();
    auto score_one = [&](int64_t u, int64_t e, int64_t r) {
        float f[kIn];
        wedge_features(A, r, e, f);
        float s = mlp_forward_row(P, f);
        s = fminf(fmaxf(s, 0.f), 30.f);
        score[u] = (double)expm1f(s);
    };
    if (wedges) {
        // listed wedges (a candidate pool): each owner by binary search over all owners
        for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += (int64_t)gridDim.x * blockDim.x) {
            const int64_t e = wedges[u];
            score_one(u, e, owner_of_f(A.fptr, A.m, e));
        }
        return;
    }
    // every wedge: the block takes 256 consecutive ones, whose owners lie between
    // the owners of its first and last (found once), and each thread searches only there
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += (int64_t)gridDim.x * blockDim.x) {
        if (threadIdx.x == 0) {
            s_own[0] = owner_of_f(A.fptr, A.m, base);
            s_own[1] = owner_of_f(A.fptr, A.m, min(base + (int64_t)blockDim.x, n) - 1);
        }
        __syncthreads();
        const int64_t u = base + threadIdx.x;
        if (u < n) {
            int64_t lo = s_own[0], hi = s_own[1] + 1;
            while (hi - lo > 1) {
                const int64_t mid = (lo + hi) >> 1;
                if (A.fptr[mid] <= u) lo = mid; else hi = mid;
            }
            score_one(u, u, lo);
        }
        __syncthreads();   // s_own is rewritten for the next chunk
    }
}

// Per row of a minibatch: forward with stored activations, then the
// backward signals.  delta = (f(x) - y) * gscale.
__global__ __launch_bounds__(256) void k_fwd_bwd_rows(const float *params, const float *x, const float *y,
                                                      const int64_t *rows, int64_t n, float gscale, float *H1,
                                                      float *H2, float *D1, float *D2, float *dout,
                                                      double *loss_parts) {
    __shared__ float P[kNumParams];
    __shared__ double lsum[256];
    for (int t = threadIdx.x; t < kNumParams; t += blockDim.x) P[t] = params[t];
    __syncthreads();
    double lacc = 0;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = rows ? rows[b] : b;
        float xr[kIn];
#pragma unroll
        for (int c = 0; c < kIn; c++) xr[c] = x[r * kIn + c];
        float h1[kH];
#pragma unroll
        for (int o = 0; o < kH; o++) {
            float z = P[kOffB1 + o];
#pragma unroll
            for (int c = 0; c < kIn; c++) z = fmaf(P[kOffW1 + o * kIn + c], xr[c], z);
            h1[o] = fmaxf(z, 0.f);
            H1[b * kH + o] = h1[o];
        }
        float out = P[kOffB3];
        for (int o = 0; o < kH; o++) {
            float z = P[kOffB2 + o];
#pragma unroll
            for (int i = 0; i < kH; i++) z = fmaf(P[kOffW2 + o * kH + i], h1[i], z);
            float h2 = fmaxf(z, 0.f);
            H2[b * kH + o] = h2;
            out = fmaf(P[kOffW3 + o], h2, out);
        }
        const float diff = out - y[r];
        lacc += 0.5 * (double)diff * (double)diff;
        const float delta = diff * gscale;
        dout[b] = delta;
        // layer-2 signals
        for (int o = 0; o < kH; o++) {
            float d2 = H2[b * kH + o] > 0.f ? delta * P[kOffW3 + o] : 0.f;
            D2[b * kH + o] = d2;
        }
        for (int i = 0; i < kH; i++) {
            float s = 0.f;
            for (int o = 0; o < kH; o++) s = fmaf(D2[b * kH + o], P[kOffW2 + o * kH + i], s);
            D1[b * kH + i] = h1[i] > 0.f ? s : 0.f;
        }
    }
    lsum[threadIdx.x] = lacc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lsum[threadIdx.x] += lsum[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_parts[blockIdx.x] = lsum[0];
}

// Parameter gradients in two fixed-order passes.  Pass 1: the rows are cut
// into chunks of `rows_per_chunk`; thread p of chunk c sums row c's
// contributions to parameter p in row order into part[c][p].  Pass 2: each
// parameter's chunk partials are summed in chunk order.  Every sum has one
// order, so the gradient is the same on every run.
__global__ void k_param_grad_parts(const float *x, const int64_t *rows, int64_t n, int64_t rows_per_chunk,
                                   const float *H1, const float *H2, const float *D1, const float *D2,
                                   const float *dout, float *part) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNumParams) return;
    const int64_t c = blockIdx.y;
    const int64_t b0 = c * rows_per_chunk;
    const int64_t b1 = b0 + rows_per_chunk < n ? b0 + rows_per_chunk : n;
    float s = 0.f;
    if (p < kOffB1) {
        const int o = p / kIn, ci = p % kIn;
        for (int64_t b = b0; b < b1; b++) {
            const int64_t r = rows ? rows[b] : b;
            s = fmaf(D1[b * kH + o], x[r * kIn + ci], s);
        }
    } else if (p < kOffW2) {
        const int o = p - kOffB1;
        for (int64_t b = b0; b < b1; b++) s += D1[b * kH + o];
    } else if (p < kOffB2) {
        const int q = p - kOffW2, o = q / kH, i = q % kH;
        for (int64_t b = b0; b < b1; b++) s = fmaf(D2[b * kH + o], H1[b * kH + i], s);
    } else if (p < kOffW3) {
        const int o = p - kOffB2;
        for (int64_t b = b0; b < b1; b++) s += D2[b * kH + o];
    } else if (p < kOffB3) {
        const int o = p - kOffW3;
        for (int64_t b = b0; b < b1; b++) s = fmaf(dout[b], H2[b * kH + o], s);
    } else {
        for (int64_t b = b0; b < b1; b++) s += dout[b];
    }
    part[c * kNumParams + p] = s;
}

__global__ void k_param_grad_sum(const float *part, int nchunks, float *grad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNumParams) return;
    float s = 0.f;
    for (int c = 0; c < nchunks; c++) s += part[(int64_t)c * kNumParams + p];
    grad[p] = s;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void k_batch_rows(uint64_t seed, uint32_t step, int64_t n, int64_t batch, int64_t *rows) {
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < batch; b += (int64_t)gridDim.x * blockDim.x)
        rows[b] = (int64_t)philox_index(seed, 16u + step, (uint64_t)b, (uint64_t)n);
}

}  // namespace

FeatArgs feat_args(Graph &g) {
    FeatArgs a;
    a.fptr = g.fptr.p;
    a.fadj = g.fadj.p;
    a.mptr = g.mptr.p;
    a.fmask = g.fmask.p;
    a.esize = g.esize.p;
    a.eptr = g.eptr.p;
    a.emem = g.emem.p;
    a.vptr = g.vptr.p;
    a.indeg = g.indeg.p;
    a.m = g.m;
    a.wbits = g.wbits;
    return a;
}

void wedge_features_all(Graph &g, float *dev_out) {
    if (g.m == 0 || g.nw == 0) return;
    hipLaunchKernelGGL(k_features_all, dim3(grid_for(g.m, 256)), dim3(256), 0, g.stream, feat_args(g), g.nw, dev_out);
    HTRI_LAUNCH_CHECK();
}

void score_wedges(Graph &g, const htri_model *model, const int64_t *dev_wedges, int64_t n, double *dev_score) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_score, dim3(grid_for(n, 256, 16384)), dim3(256), 0, g.stream, feat_args(g),
                       model->params.p, dev_wedges, n, dev_score);
    HTRI_LAUNCH_CHECK();
}

namespace {

// loss and gradient over rows (all n rows, or a minibatch given by `rows`)
constexpr int64_t kGradRowsPerChunk = 64;
constexpr int64_t kGradMaxChunks = 512;

struct GradBufs {
    DBuf<float> H1, H2, D1, D2, dout, part;
    DBuf<double> lp;
    int grid = 1;
    GradBufs(Allocator &A, int64_t n) : H1(A, n * kH), H2(A, n * kH), D1(A, n * kH), D2(A, n * kH), dout(A, n) {
        grid = (int)std::min<int64_t>((n + 255) / 256, 4096);
        if (grid < 1) grid = 1;
        lp.alloc(A, grid);
        part.alloc(A, (size_t)kGradMaxChunks * kNumParams);
    }
};

// rows per chunk and chunk count of the gradient's first pass for n rows
inline void grad_chunks(int64_t n, int64_t &rows_per_chunk, int &nchunks) {
    rows_per_chunk = std::max<int64_t>(kGradRowsPerChunk, (n + kGradMaxChunks - 1) / kGradMaxChunks);
    nchunks = (int)std::max<int64_t>(1, (n + rows_per_chunk - 1) / rows_per_chunk);
}

double loss_grad(htri_model *mdl, GradBufs &B, const float *x, const float *y, const int64_t *rows, int64_t n,
                 float *grad_dev) {
    hipStream_t s = mdl->stream;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, B.grid);
    hipLaunchKernelGGL(k_fwd_bwd_rows, dim3(grid), dim3(256), 0, s, mdl->params.p, x, y, rows, n, 1.0f / (float)n,
                       B.H1.p, B.H2.p, B.D1.p, B.D2.p, B.dout.p, B.lp.p);
    HTRI_LAUNCH_CHECK();
    int64_t rpc;
    int nch;
    grad_chunks(n, rpc, nch);
    hipLaunchKernelGGL(k_param_grad_parts, dim3((kNumParams + 255) / 256, nch), dim3(256), 0, s, x, rows, n, rpc,
                       B.H1.p, B.H2.p, B.D1.p, B.D2.p, B.dout.p, B.part.p);
    HTRI_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_param_grad_sum, dim3((kNumParams + 255) / 256), dim3(256), 0, s, B.part.p, nch, grad_dev);
    HTRI_LAUNCH_CHECK();
    std::vector<double> h(grid);
    HTRI_HIP(hipMemcpyAsync(h.data(), B.lp.p, sizeof(double) * grid, hipMemcpyDeviceToHost, s));
    HTRI_HIP(hipStreamSynchronize(s));
    double L = 0;
    for (double v : h) L += v;
    return L / (double)n;
}

}  // namespace

}  // namespace htri

using namespace htri;

namespace {
template <typename F>
htri_status run_model(htri_model *m, F &&fn) {
    try {
        fn();
        return HTRI_OK;
    } catch (const htri::Error &e) {
        if (m) m->err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        return HTRI_E_OOM;
    }
}
}  // namespace

extern "C" {

htri_status htri_model_create(uint64_t seed, void *stream, htri_model **out) {
    if (!out) return HTRI_E_INVALID;
    *out = nullptr;
    htri_model *m = new (std::nothrow) htri_model();
    if (!m) return HTRI_E_OOM;
    m->stream = (hipStream_t)stream;
    m->al.stream = (hipStream_t)stream;
    htri_status st = run_model(m, [&] {
        m->params.alloc(m->al, kNumParams);
        m->adam_m.alloc(m->al, kNumParams);
        m->adam_v.alloc(m->al, kNumParams);
        // He-uniform initialisation from a Philox stream, zero biases
        std::vector<float> p(kNumParams, 0.f);
        auto fill = [&](int off, int count, int fan_in) {
            const double bound = std::sqrt(6.0 / fan_in);
            for (int i = 0; i < count; i++) p[off + i] = (float)((2.0 * philox_unit(seed, 7u, (uint64_t)(off + i)) - 1.0) * bound);
        };
        fill(kOffW1, kH * kIn, kIn);
        fill(kOffW2, kH * kH, kH);
        fill(kOffW3, kH, kH);
        HTRI_HIP(hipMemcpyAsync(m->params.p, p.data(), sizeof(float) * kNumParams, hipMemcpyHostToDevice, m->stream));
        fill_u32((uint32_t *)m->adam_m.p, kNumParams, 0, m->stream);
        fill_u32((uint32_t *)m->adam_v.p, kNumParams, 0, m->stream);
        HTRI_HIP(hipStreamSynchronize(m->stream));
    });
    if (st != HTRI_OK) {
        delete m;
        return st;
    }
    *out = m;
    return HTRI_OK;
}

void htri_model_free(htri_model *m) {
    if (!m) return;
    (void)hipStreamSynchronize(m->stream);
    delete m;
}

htri_status htri_model_get_params(const htri_model *mc, float *host_params) {
    htri_model *m = const_cast<htri_model *>(mc);
    if (!m || !host_params) return HTRI_E_INVALID;
    return run_model(m, [&] {
        HTRI_HIP(hipMemcpyAsync(host_params, m->params.p, sizeof(float) * kNumParams, hipMemcpyDeviceToHost, m->stream));
        HTRI_HIP(hipStreamSynchronize(m->stream));
    });
}

htri_status htri_model_set_params(htri_model *m, const float *host_params) {
    if (!m || !host_params) return HTRI_E_INVALID;
    return run_model(m, [&] {
        HTRI_HIP(hipMemcpyAsync(m->params.p, host_params, sizeof(float) * kNumParams, hipMemcpyHostToDevice, m->stream));
        fill_u32((uint32_t *)m->adam_m.p, kNumParams, 0, m->stream);
        fill_u32((uint32_t *)m->adam_v.p, kNumParams, 0, m->stream);
        m->adam_t = 0;
        HTRI_HIP(hipStreamSynchronize(m->stream));
    });
}

// Metadata written beside the raw parameters; a load accepts only files whose
// metadata names this layout.
static const char kModelMeta[] =
    "{\"format\": \"htri-proposal-mlp\", \"version\": 1, \"layers\": [16, 64, 64, 1], "
    "\"activation\": \"relu\", \"dtype\": \"float32\", \"byte_order\": \"little\", "
    "\"num_params\": 5313, \"layout\": [\"W1[64][16]\", \"b1[64]\", \"W2[64][64]\", \"b2[64]\", "
    "\"w3[64]\", \"b3\"]}\n";

const char *htri_model_last_error(const htri_model *m) { return m ? m->err.c_str() : ""; }

htri_status htri_model_save(const htri_model *mc, const char *path) {
    htri_model *m = const_cast<htri_model *>(mc);
    if (!m || !path || !*path) return HTRI_E_INVALID;
    std::vector<float> p(kNumParams);
    htri_status st = htri_model_get_params(m, p.data());
    if (st != HTRI_OK) return st;
    const std::string meta = std::string(path) + ".json";
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        m->err = std::string("cannot open ") + path + " for writing";
        return HTRI_E_INVALID;
    }
    const bool ok = std::fwrite(p.data(), sizeof(float), kNumParams, f) == (size_t)kNumParams;
    if (std::fclose(f) != 0 || !ok) {
        m->err = std::string("short write to ") + path;
        return HTRI_E_INVALID;
    }
    FILE *j = std::fopen(meta.c_str(), "wb");
    if (!j) {
        m->err = "cannot open " + meta + " for writing";
        return HTRI_E_INVALID;
    }
    const size_t len = sizeof(kModelMeta) - 1;
    const bool ok2 = std::fwrite(kModelMeta, 1, len, j) == len;
    if (std::fclose(j) != 0 || !ok2) {
        m->err = "short write to " + meta;
        return HTRI_E_INVALID;
    }
    return HTRI_OK;
}

htri_status htri_model_load(htri_model *m, const char *path) {
    if (!m || !path || !*path) return HTRI_E_INVALID;
    const std::string meta = std::string(path) + ".json";
    FILE *j = std::fopen(meta.c_str(), "rb");
    if (!j) {
        m->err = "cannot open " + meta;
        return HTRI_E_INVALID;
    }
    std::string text;
    char buf[512];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof(buf), j)) > 0 && text.size() < 65536) text.append(buf, got);
    std::fclose(j);
    if (text.find("\"htri-proposal-mlp\"") == std::string::npos ||
        text.find("\"num_params\": 5313") == std::string::npos ||
        text.find("\"float32\"") == std::string::npos) {
        m->err = meta + " does not describe a 16-64-64-1 float32 proposal network";
        return HTRI_E_INVALID;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        m->err = std::string("cannot open ") + path;
        return HTRI_E_INVALID;
    }
    std::vector<float> p(kNumParams + 1);
    const size_t n = std::fread(p.data(), sizeof(float), kNumParams + 1, f);
    std::fclose(f);
    if (n != (size_t)kNumParams) {
        m->err = std::string(path) + " does not hold exactly 5313 float32 parameters";
        return HTRI_E_INVALID;
    }
    for (int i = 0; i < kNumParams; i++)
        if (!std::isfinite(p[i])) {
            m->err = std::string(path) + " holds a non-finite parameter";
            return HTRI_E_INVALID;
        }
    return htri_model_set_params(m, p.data());
}

htri_status htri_model_forward(const htri_model *mc, const float *dev_x, int64_t n, float *dev_out) {
    htri_model *m = const_cast<htri_model *>(mc);
    if (!m || n < 0 || (n > 0 && (!dev_x || !dev_out))) return HTRI_E_INVALID;
    return run_model(m, [&] {
        if (n == 0) return;
        hipLaunchKernelGGL(k_forward, dim3(grid_for(n, 256, 16384)), dim3(256), 0, m->stream, m->params.p, dev_x, n,
                           dev_out);
        HTRI_LAUNCH_CHECK();
        HTRI_HIP(hipStreamSynchronize(m->stream));
    });
}

htri_status htri_model_loss_grad(const htri_model *mc, const float *dev_x, const float *dev_y, int64_t n,
                                 double *loss, float *host_grad) {
    htri_model *m = const_cast<htri_model *>(mc);
    if (!m || n <= 0 || !dev_x || !dev_y || !loss || !host_grad) return HTRI_E_INVALID;
    return run_model(m, [&] {
        DBuf<float> g(m->al, kNumParams);
        GradBufs B(m->al, n);
        *loss = loss_grad(m, B, dev_x, dev_y, nullptr, n, g.p);
        HTRI_HIP(hipMemcpyAsync(host_grad, g.p, sizeof(float) * kNumParams, hipMemcpyDeviceToHost, m->stream));
        HTRI_HIP(hipStreamSynchronize(m->stream));
    });
}

htri_status htri_model_train(htri_model *m, const float *dev_x, const float *dev_y, int64_t n, int32_t steps,
                             int32_t batch, float lr, uint64_t seed, double *final_loss) {
    if (!m || n <= 0 || steps < 0 || batch <= 0 || !dev_x || !dev_y) return HTRI_E_INVALID;
    return run_model(m, [&] {
        DBuf<int64_t> rows(m->al, batch);
        DBuf<float> g(m->al, kNumParams);
        GradBufs B(m->al, batch);
        double L = 0;
        const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
        for (int32_t st = 0; st < steps; st++) {
            hipLaunchKernelGGL(k_batch_rows, dim3(grid_for(batch, 256)), dim3(256), 0, m->stream, seed, (uint32_t)st, n,
                               (int64_t)batch, rows.p);
            HTRI_LAUNCH_CHECK();
            L = loss_grad(m, B, dev_x, dev_y, rows.p, batch, g.p);
            m->adam_t++;
            const float c1 = 1.f - std::pow(b1, (float)m->adam_t), c2 = 1.f - std::pow(b2, (float)m->adam_t);
            hipLaunchKernelGGL(k_adam, dim3((kNumParams + 255) / 256), dim3(256), 0, m->stream, m->params.p, g.p,
                               m->adam_m.p, m->adam_v.p, kNumParams, lr, b1, b2, eps, c1, c2);
            HTRI_LAUNCH_CHECK();
        }
        HTRI_HIP(hipStreamSynchronize(m->stream));
        if (final_loss) *final_loss = L;
    });
}

}  // extern "C"

// Learned start proposal: a small network predicts where a foot lies in a
// chart of the mesh, a table turns the chart position into a start triangle,
// and the exact walk finishes the search.  The element found never depends
// on the network (the walk's result does not depend on its start); the
// network only shortens walks.  This develops the remark closing the
// numerical section (Section 4) on choosing the walk's start from local
// information about the dynamics.
//
// Chart: Rosenblatt coordinates of the triangle centroids, u = F_x(x) (rank
// of the centroid's x) and v = F_{y|u}(y) (rank of its y within its u slab),
// so that equal chart areas hold equal numbers of triangles whatever the
// grading.  The G x G table maps a chart cell to the triangle whose chart
// centroid is nearest the cell centre (empty cells: the nearest filled cell).
//
// Network: (x, y, dx, dy, t) -> 64 -> 64 -> 2 with ReLU, regressing the chart
// displacement from the node to the element that contains its foot (dx, dy =
// foot - node): the proposal is chart(node) + output, so the network never
// has to rebuild the chart itself, only how far the foot moves in it.
// The exact chart cell of a foot (two binary searches in quantile tables,
// no network) is the non-learned form of the same start.
// Training: FP32 forward and backward kernels, per-workgroup partial
// gradients summed in a fixed order (bit-reproducible), Adam.  Inference:
// bfloat16 operands on the matrix cores, FP32 accumulation (slw_mlp.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <deque>
#include <new>
#include <numeric>
#include <vector>

#include "slw_internal.h"
#include "slw_mlp.h"

namespace slw {
namespace {

constexpr int kBlock = 256;
constexpr int kPartialStride = kMlpParams + 2;  // gradient, loss sum, valid count
constexpr int kOwned = 74;                      // gradient entries each lane accumulates

// sample order of an epoch: i -> (a i + c) mod m, a coprime to m
__device__ inline int64_t perm_index(int64_t i, int64_t m, uint64_t a, uint64_t c)
{
    return (int64_t)(((unsigned __int128)a * (uint64_t)i + c) % (uint64_t)m);
}

// Partial gradient of the mean squared error over the samples [first,
// first + count) of the epoch order, split evenly over the workgroups (one
// wavefront each).  Per 64 samples: forward and backward one lane per sample,
// activations and deltas staged in LDS, then each lane accumulates the
// gradient entries it owns over the 64 samples (dW1[.][t], db1[t], dW2[.][t],
// db2[t], two entries of dW3, db3[t] for t < 2).  Samples whose target is
// NaN (foot outside) count in the batch size but carry no error.
__global__ void __launch_bounds__(64)
    k_mlp_partial(const float *__restrict__ P, const float *__restrict__ norm, const float *__restrict__ X,
                  const float2 *__restrict__ Y, int64_t m, int64_t first, int64_t count, uint64_t pa, uint64_t pc,
                  float inv_batch, float *__restrict__ partial)
{
    __shared__ float sX[64][5];
    __shared__ float sA[64][65];  // h1, then delta1 (row = sample; odd stride: no bank conflicts)
    __shared__ float sB[64][65];  // h2, then delta2
    __shared__ float sD3[64][2];
    __shared__ float sG[kOwned][64];
    const int t = threadIdx.x;
    const int64_t per = (count + gridDim.x - 1) / gridDim.x;
    const int64_t lo = first + (int64_t)blockIdx.x * per;
    const int64_t hi = min(first + count, lo + per);
    for (int k = 0; k < kOwned; ++k)
        sG[k][t] = 0.f;
    float loss = 0.f, valid = 0.f;
    for (int64_t c0 = lo; c0 < hi; c0 += 64) {
        const int64_t i = c0 + t;
        float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f}, y0 = 0.f, y1 = 0.f, w = 0.f;
        if (i < hi) {
            const int64_t s = perm_index(i, m, pa, pc);
#pragma unroll
            for (int c = 0; c < 5; ++c)
                x[c] = X[5 * s + c];
            mlp_normalise(norm, x);
            const float2 yy = Y[s];
            if (yy.x == yy.x) {  // NaN: no target
                y0 = yy.x;
                y1 = yy.y;
                w = 1.f;
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c)
            sX[t][c] = x[c];
        // forward (padding lanes carry w = 0: their deltas vanish)
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            float z = P[kOB1 + j];
#pragma unroll
            for (int c = 0; c < 5; ++c)
                z = fmaf(x[c], P[kOW1 + c * 64 + j], z);
            sA[t][j] = fmaxf(z, 0.f);
        }
        // layer 2 with the weights read row by row (contiguous, uniform:
        // wide scalar loads), inputs from LDS, 64 accumulators in registers
        float z2[64];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            z2[j] = P[kOB2 + j];
        for (int c = 0; c < 64; ++c) {
            const float hc = sA[t][c];
#pragma unroll
            for (int j = 0; j < 64; ++j)
                z2[j] = fmaf(hc, P[kOW2 + c * 64 + j], z2[j]);
        }
        float o0 = P[kOB3], o1 = P[kOB3 + 1];
#pragma unroll
        for (int j = 0; j < 64; ++j) {
            const float h2 = fmaxf(z2[j], 0.f);
            sB[t][j] = h2;
            o0 = fmaf(h2, P[kOW3 + 2 * j], o0);
            o1 = fmaf(h2, P[kOW3 + 2 * j + 1], o1);
        }
        const float e0 = o0 - y0, e1 = o1 - y1;
        loss += w * (e0 * e0 + e1 * e1);
        valid += w;
        const float d30 = 2.f * e0 * w * inv_batch, d31 = 2.f * e1 * w * inv_batch;
        sD3[t][0] = d30;
        sD3[t][1] = d31;
        __syncthreads();
        // dW3 entries t and 64 + t: (i, j) = (t / 2, t % 2) and (32 + t / 2, t % 2); db3
        {
            const int i0 = t >> 1, jj = t & 1;
            float s0 = 0.f, s1 = 0.f, sb = 0.f;
            for (int s = 0; s < 64; ++s) {
                s0 = fmaf(sB[s][i0], sD3[s][jj], s0);
                s1 = fmaf(sB[s][32 + i0], sD3[s][jj], s1);
                sb += sD3[s][jj];
            }
            sG[71][t] += s0;
            sG[72][t] += s1;
            if (t < 2)
                sG[73][t] += sb;
        }
        __syncthreads();
        // delta2 = (delta3 W3^T) masked by h2 > 0, over h2 in LDS (own row)
        for (int j = 0; j < 64; ++j) {
            const float h2 = sB[t][j];
            sB[t][j] = h2 > 0.f ? fmaf(d30, P[kOW3 + 2 * j], d31 * P[kOW3 + 2 * j + 1]) : 0.f;
        }
        __syncthreads();
        // dW2[k][t] = sum_s h1[s][k] delta2[s][t]; db2[t]
        for (int k = 0; k < 64; ++k) {
            float s2 = 0.f;
            for (int s = 0; s < 64; ++s)
                s2 = fmaf(sA[s][k], sB[s][t], s2);
            sG[6 + k][t] += s2;
        }
        {
            float sb2 = 0.f;
            for (int s = 0; s < 64; ++s)
                sb2 += sB[s][t];
            sG[70][t] += sb2;
        }
        __syncthreads();
        // delta1 = (delta2 W2^T) masked by h1 > 0, over h1 in LDS (own row);
        // delta2 in registers, weight rows contiguous
        float d2[64];
#pragma unroll
        for (int j = 0; j < 64; ++j)
            d2[j] = sB[t][j];
        for (int c = 0; c < 64; ++c) {
            float z = 0.f;
#pragma unroll
            for (int j = 0; j < 64; ++j)
                z = fmaf(d2[j], P[kOW2 + c * 64 + j], z);
            const float h = sA[t][c];
            sA[t][c] = h > 0.f ? z : 0.f;
        }
        __syncthreads();
        // dW1[k][t] = sum_s x[s][k] delta1[s][t]; db1[t]
        for (int k = 0; k < 5; ++k) {
            float s1 = 0.f;
            for (int s = 0; s < 64; ++s)
                s1 = fmaf(sX[s][k], sA[s][t], s1);
            sG[k][t] += s1;
        }
        {
            float sb1 = 0.f;
            for (int s = 0; s < 64; ++s)
                sb1 += sA[s][t];
            sG[5][t] += sb1;
        }
        __syncthreads();
    }
    float *out = partial + (int64_t)blockIdx.x * kPartialStride;
    for (int k = 0; k < 5; ++k)
        out[kOW1 + k * 64 + t] = sG[k][t];
    out[kOB1 + t] = sG[5][t];
    for (int k = 0; k < 64; ++k)
        out[kOW2 + k * 64 + t] = sG[6 + k][t];
    out[kOB2 + t] = sG[70][t];
    out[kOW3 + t] = sG[71][t];
    out[kOW3 + 64 + t] = sG[72][t];
    if (t < 2)
        out[kOB3 + t] = sG[73][t];
    for (int off = 32; off > 0; off >>= 1) {
        loss += __shfl_xor(loss, off, 64);
        valid += __shfl_xor(valid, off, 64);
    }
    if (t == 0) {
        out[kMlpParams] = loss;
        out[kMlpParams + 1] = valid;
    }
}

// out[e] = sum over workgroups b, in order, of partial[b][e]
// Sum of the nb partial gradients, entry by entry, in a fixed order: a
// workgroup takes 64 consecutive entries; its 4 wavefronts each add every
// 4th partial (8 loads in flight per lane), then the four sums are added in
// wavefront order.
__global__ void __launch_bounds__(256) k_mlp_reduce(const float *__restrict__ partial, int nb, float *__restrict__ out,
                                                    int n)
{
    __shared__ float s4[4][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (e < n) {
        int b = wv;
        for (; b + 28 < nb; b += 32) {
            float v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                v[u] = partial[(int64_t)(b + 4 * u) * kPartialStride + e];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                s += v[u];
        }
        for (; b < nb; b += 4)
            s += partial[(int64_t)b * kPartialStride + e];
    }
    s4[wv][lane] = s;
    __syncthreads();
    if (wv == 0 && e < n)
        out[e] = ((s4[0][lane] + s4[1][lane]) + s4[2][lane]) + s4[3][lane];
}

// Adam with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n)
        return;
    const float ge = g[e];
    const float mm = b1 * m[e] + (1.f - b1) * ge;
    const float vv = b2 * v[e] + (1.f - b2) * ge * ge;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// bfloat16 operands in the per-lane layout of mlp_forward_wave, biases in
// accumulator order
__global__ void k_mlp_pack(const float *__restrict__ P, uint16_t *__restrict__ wpack, float *__restrict__ bias)
{
    const int l = threadIdx.x;  // 64 lanes
    const int grp = l >> 4, col = l & 15;
    for (int mt = 0; mt < 4; ++mt)  // A[i][k] = W1[k][16 mt + i]
        for (int c = 0; c < 4; ++c) {
            const int k = 4 * grp + c;
            wpack[(mt * 64 + l) * 4 + c] = to_bf16(k < 5 ? P[kOW1 + k * 64 + 16 * mt + col] : 0.f);
        }
    for (int mt2 = 0; mt2 < 4; ++mt2)  // A[i][k] = W2[16 kk + k][16 mt2 + i]
        for (int kk = 0; kk < 4; ++kk)
            for (int c = 0; c < 4; ++c)
                wpack[4 * 64 * 4 + ((mt2 * 4 + kk) * 64 + l) * 4 + c] =
                    to_bf16(P[kOW2 + (16 * kk + 4 * grp + c) * 64 + 16 * mt2 + col]);
    for (int kk = 0; kk < 4; ++kk)  // A[i][k] = W3[16 kk + k][i] for i < 2
        for (int c = 0; c < 4; ++c)
            wpack[20 * 64 * 4 + (kk * 64 + l) * 4 + c] =
                to_bf16(col < 2 ? P[kOW3 + (16 * kk + 4 * grp + c) * 2 + col] : 0.f);
    bias[l] = P[kOB1 + l];
    bias[64 + l] = P[kOB2 + l];
    if (l < 16)
        bias[128 + l] = l < 2 ? P[kOB3 + l] : 0.f;
}

// the network on given raw features: out[i] = outputs of X[i]
__global__ void __launch_bounds__(kBlock)
    k_mlp_forward(const uint16_t *__restrict__ wpack, const float *__restrict__ bias, const float *__restrict__ norm,
                  const float *__restrict__ X, int64_t m, float2 *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    float feat[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < m) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
            feat[c] = X[5 * i + c];
        mlp_normalise(norm, feat);
    }
    const float2 uv = mlp_forward_wave(wpack, bias, feat);  // every lane
    if (i < m)
        out[i] = uv;
}

// feature means and inverse standard deviations: per-workgroup FP64 sums of
// x and x^2 of every feature over a contiguous slice of the samples
// (kNormParts workgroups), then one workgroup adds the partial sums in a
// fixed order (bit-reproducible)
constexpr int kNormParts = 512;
__global__ void __launch_bounds__(kBlock) k_fit_norm_partial(const float *__restrict__ X, int64_t m,
                                                             double *__restrict__ part)
{
    __shared__ double s[10][kBlock];
    const int64_t per = (m + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(m, lo + per);
    double a[5] = {0, 0, 0, 0, 0}, b[5] = {0, 0, 0, 0, 0};
    for (int64_t i = lo + threadIdx.x; i < hi; i += kBlock) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const double x = X[5 * i + c];
            a[c] += x;
            b[c] += x * x;
        }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        s[c][threadIdx.x] = a[c];
        s[5 + c][threadIdx.x] = b[c];
    }
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
#pragma unroll
            for (int c = 0; c < 10; ++c)
                s[c][threadIdx.x] += s[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 10)
        part[10 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) k_fit_norm_final(const double *__restrict__ part, int parts, int64_t m,
                                                       float *__restrict__ norm)
{
    const int c = threadIdx.x;
    if (c >= 5)
        return;
    double a = 0.0, b = 0.0;
    for (int p = 0; p < parts; ++p) {
        a += part[10 * p + c];
        b += part[10 * p + 5 + c];
    }
    const double mean = m > 0 ? a / (double)m : 0.0;
    const double var = m > 0 ? fmax(b / (double)m - mean * mean, 0.0) : 0.0;
    norm[c] = (float)mean;
    norm[5 + c] = var > 0.0 ? (float)(1.0 / sqrt(var)) : 1.0f;
}

uint64_t splitmix64(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

slw_status mlp_pack(slw_mlp *n)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(1), dim3(64), 0, n->ctx->stream, n->params, n->wpack, n->bias);
    return hip_check(hipGetLastError(), "pack network weights");
}

slw_status gradient_pass(slw_mlp *n, const float *X, const float *Y, int64_t m, int64_t first, int64_t count,
                         uint64_t pa, uint64_t pc, float inv_batch)
{
    hipStream_t st = n->ctx->stream;
    // about 64 samples per workgroup, at most kMlpPartials workgroups (a
    // function of count only: the sums stay bit-reproducible); minibatches
    // of 65,536 samples fill the device
    const int nb = (int)std::min<int64_t>(kMlpPartials, std::max<int64_t>(1, (count + 63) / 64));
    hipLaunchKernelGGL(k_mlp_partial, dim3(nb), dim3(64), 0, st, n->params, n->norm, X, (const float2 *)Y, m, first,
                       count, pa, pc, inv_batch, n->partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_check(e, "gradient partials");
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kPartialStride + 63) / 64), dim3(256), 0, st, n->partial, nb, n->grad,
                       kPartialStride);
    return hip_check(hipGetLastError(), "gradient reduction");
}

// mean squared error of the last gradient pass over its valid samples
slw_status read_loss(slw_mlp *n, float *loss_h)
{
    float lv[2];
    slw_status st = hip_check(hipMemcpyAsync(lv, n->grad + kMlpParams, sizeof lv, hipMemcpyDeviceToHost,
                                             n->ctx->stream),
                              "copy loss");
    if (st == SLW_OK)
        st = hip_check(hipStreamSynchronize(n->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK && loss_h)
        *loss_h = lv[1] > 0.f ? lv[0] / lv[1] : 0.f;
    return st;
}

}  // namespace
}  // namespace slw

using namespace slw;

extern "C" {

slw_status slw_chart_build(slw_mesh *mesh, int g)
{
    if (!mesh || g < 1 || g > 8192)
        return set_error(SLW_E_ARG, "slw_chart_build: null mesh or g outside [1, 8192]");
    DevMesh &m = mesh->m;
    DeviceGuard gd(mesh->ctx->device);
    const int64_t nt = m.n_tris, nd = m.n_dofs;
    std::vector<GeoRec> geo(nt);
    slw_status st = hip_check(hipStreamSynchronize(mesh->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(geo.data(), m.geo, nt * sizeof(GeoRec), hipMemcpyDeviceToHost), "copy records");
    if (st != SLW_OK)
        return st;
    // Everything in the records' float frame (coordinates minus the centre
    // used at upload): centroids, DOF positions, and the feet of the lookup.
    std::vector<float> cx(nt), cy(nt);
    for (int64_t t = 0; t < nt; ++t) {
        cx[t] = (float)(((double)geo[t].p[0].x + geo[t].p[1].x + geo[t].p[2].x) / 3.0);
        cy[t] = (float)(((double)geo[t].p[0].y + geo[t].p[1].y + geo[t].p[2].y) / 3.0);
    }
    // u: rank of the centroid's x; slab = floor(u g); v: rank of y in the slab
    std::vector<int32_t> ord(nt);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return cx[a] != cx[b] ? cx[a] < cx[b] : a < b; });
    std::vector<float2> uv(nt);
    std::vector<std::vector<int32_t>> slab(g);
    std::vector<float> qx(g, INFINITY);  // smallest centroid x of each slab
    for (int64_t r = 0; r < nt; ++r) {
        const double u = ((double)r + 0.5) / (double)nt;
        const int s = (int)std::min<int64_t>(g - 1, (int64_t)(u * g));
        uv[ord[r]].x = (float)u;
        if (slab[s].empty())
            qx[s] = cx[ord[r]];
        slab[s].push_back(ord[r]);
    }
    std::vector<float> qy((size_t)g * g, INFINITY);  // smallest centroid y of each cell of a slab
    std::vector<std::vector<float>> ys(g);           // sorted centroid y of each slab
    for (int s = 0; s < g; ++s) {
        auto &v = slab[s];
        std::sort(v.begin(), v.end(), [&](int32_t a, int32_t b) { return cy[a] != cy[b] ? cy[a] < cy[b] : a < b; });
        ys[s].resize(v.size());
        for (size_t r = 0; r < v.size(); ++r) {
            const double vv = ((double)r + 0.5) / (double)v.size();
            const int j = (int)std::min<int64_t>(g - 1, (int64_t)(vv * g));
            uv[v[r]].y = (float)vv;
            ys[s][r] = cy[v[r]];
            float &q = qy[(size_t)s * g + j];
            q = std::min(q, cy[v[r]]);
        }
    }
    // empty slabs / cells take the next threshold, so the tables stay sorted
    for (int s = g - 2; s >= 0; --s)
        qx[s] = std::min(qx[s], qx[s + 1]);
    for (int s = 0; s < g; ++s)
        for (int j = g - 2; j >= 0; --j)
            qy[(size_t)s * g + j] = std::min(qy[(size_t)s * g + j], qy[(size_t)s * g + j + 1]);
    // chart coordinates of the DOFs: the same ranks for their positions
    std::vector<float> sx(nt);
    for (int64_t r = 0; r < nt; ++r)
        sx[r] = cx[ord[r]];
    std::vector<float2> node(std::max<int64_t>(nd, 1));
    for (int64_t d = 0; d < nd; ++d) {
        const int64_t du = m.dof_user_h[d];
        const float px = (float)(m.dof_xy_user_h[2 * du] - m.fc.cx), py = (float)(m.dof_xy_user_h[2 * du + 1] - m.fc.cy);
        const double u = (double)(std::lower_bound(sx.begin(), sx.end(), px) - sx.begin()) / (double)nt;
        const int s = (int)std::min<int64_t>(g - 1, (int64_t)(u * g));
        const auto &y = ys[s];
        const double v = y.empty() ? 0.5 : (double)(std::lower_bound(y.begin(), y.end(), py) - y.begin()) / y.size();
        node[d] = make_float2((float)u, (float)v);
    }
    // cell -> triangle whose chart centroid is nearest the cell centre
    std::vector<int32_t> table((size_t)g * g, -1);
    std::vector<float> best((size_t)g * g, INFINITY);
    for (int64_t t = 0; t < nt; ++t) {
        const int bu = std::min(g - 1, (int)(uv[t].x * (float)g)), bv = std::min(g - 1, (int)(uv[t].y * (float)g));
        const float du = uv[t].x * g - (bu + 0.5f), dv = uv[t].y * g - (bv + 0.5f);
        const float d2 = du * du + dv * dv;
        const size_t c = (size_t)bu * g + bv;
        if (d2 < best[c]) {
            best[c] = d2;
            table[c] = (int32_t)t;
        }
    }
    // empty cells: breadth-first fill from the filled ones
    std::deque<size_t> qu;
    for (size_t c = 0; c < table.size(); ++c)
        if (table[c] >= 0)
            qu.push_back(c);
    while (!qu.empty()) {
        const size_t c = qu.front();
        qu.pop_front();
        const int bu = (int)(c / g), bv = (int)(c % g);
        const int du[4] = {1, -1, 0, 0}, dv[4] = {0, 0, 1, -1};
        for (int s = 0; s < 4; ++s) {
            const int nu = bu + du[s], nv = bv + dv[s];
            if (nu < 0 || nv < 0 || nu >= g || nv >= g)
                continue;
            const size_t nc = (size_t)nu * g + nv;
            if (table[nc] < 0) {
                table[nc] = table[c];
                qu.push_back(nc);
            }
        }
    }
    // device copies (the old chart is replaced only when all succeeded)
    const size_t gg = (size_t)g * g;
    float2 *uv_d = nullptr, *node_d = nullptr;
    int32_t *tab_d = nullptr, *start_d = nullptr;
    float *qx_d = nullptr, *qy_d = nullptr;
    bool ok = hipMalloc((void **)&uv_d, std::max<int64_t>(nt, 1) * sizeof(float2)) == hipSuccess &&
              hipMalloc((void **)&node_d, node.size() * sizeof(float2)) == hipSuccess &&
              hipMalloc((void **)&tab_d, gg * sizeof(int32_t)) == hipSuccess &&
              hipMalloc((void **)&qx_d, g * sizeof(float)) == hipSuccess &&
              hipMalloc((void **)&qy_d, gg * sizeof(float)) == hipSuccess &&
              (m.learned_start ||
               hipMalloc((void **)&start_d, std::max<int64_t>(nd, 1) * sizeof(int32_t)) == hipSuccess);
    if (ok) {
        ok = hipMemcpy(uv_d, uv.data(), nt * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(node_d, node.data(), node.size() * sizeof(float2), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(tab_d, table.data(), gg * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(qx_d, qx.data(), g * sizeof(float), hipMemcpyHostToDevice) == hipSuccess &&
             hipMemcpy(qy_d, qy.data(), gg * sizeof(float), hipMemcpyHostToDevice) == hipSuccess;
        if (!ok)
            st = set_error(SLW_E_HIP, "slw_chart_build: copy to the device");
    } else {
        st = set_error(SLW_E_NOMEM, "slw_chart_build: chart arrays");
    }
    if (!ok) {
        void *p[] = {uv_d, node_d, tab_d, qx_d, qy_d, start_d};
        for (void *q : p)
            if (q)
                (void)hipFree(q);
        return st;
    }
    void *old[] = {m.chart_uv, m.chart_node, m.chart_table, m.chart_qx, m.chart_qy};
    for (void *q : old)
        if (q)
            (void)hipFree(q);
    const int64_t old_bytes = m.chart_g ? nt * 8 + nd * 8 + (int64_t)m.chart_g * (8 * m.chart_g + 4) : 0;
    m.device_bytes += nt * 8 + nd * 8 + (int64_t)g * (8 * g + 4) - old_bytes;
    if (start_d) {
        m.learned_start = start_d;
        m.device_bytes += std::max<int64_t>(nd, 1) * 4;
    }
    m.chart_uv = uv_d;
    m.chart_node = node_d;
    m.chart_table = tab_d;
    m.chart_qx = qx_d;
    m.chart_qy = qy_d;
    m.chart_g = g;
    return SLW_OK;
}

slw_status slw_chart_coords(slw_mesh *mesh, float *uv_h)
{
    if (!mesh || !uv_h)
        return set_error(SLW_E_ARG, "slw_chart_coords: null pointer");
    const DevMesh &m = mesh->m;
    if (!m.chart_uv)
        return set_error(SLW_E_ARG, "slw_chart_coords: no chart (slw_chart_build)");
    DeviceGuard gd(mesh->ctx->device);
    std::vector<float2> uv(m.n_tris);
    std::vector<int32_t> uf(m.n_tris);
    slw_status st = hip_check(hipStreamSynchronize(mesh->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(uv.data(), m.chart_uv, uv.size() * sizeof(float2), hipMemcpyDeviceToHost),
                       "copy chart");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(uf.data(), m.tri_uf, uf.size() * sizeof(int32_t), hipMemcpyDeviceToHost),
                       "copy ids");
    if (st != SLW_OK)
        return st;
    for (int64_t t = 0; t < m.n_tris; ++t) {
        const int64_t u = uf[t] & 0x7fffffff;
        uv_h[2 * u] = uv[t].x;
        uv_h[2 * u + 1] = uv[t].y;
    }
    return SLW_OK;
}

slw_status slw_mlp_create(slw_ctx *ctx, uint64_t seed, slw_mlp **out)
{
    if (!ctx || !out)
        return set_error(SLW_E_ARG, "slw_mlp_create: null pointer");
    *out = nullptr;
    DeviceGuard gd(ctx->device);
    slw_mlp *n = new (std::nothrow) slw_mlp();
    if (!n)
        return set_error(SLW_E_NOMEM, "network");
    n->ctx = ctx;
    const bool ok =
        hipMalloc((void **)&n->params, kMlpParams * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->adam_m, kMlpParams * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->adam_v, kMlpParams * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->grad, kPartialStride * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->partial, (size_t)kMlpPartials * kPartialStride * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->norm, 10 * sizeof(float)) == hipSuccess &&
        hipMalloc((void **)&n->wpack, kWpackHalves * sizeof(uint16_t)) == hipSuccess &&
        hipMalloc((void **)&n->bias, kBiasFloats * sizeof(float)) == hipSuccess;
    if (!ok) {
        slw_mlp_free(n);
        return set_error(SLW_E_NOMEM, "network buffers");
    }
    // He-uniform weights (limit sqrt(6 / fan_in)) from a splitmix64 stream, zero biases
    std::vector<float> p(kMlpParams, 0.f);
    uint64_t s = seed;
    auto uni = [&](double lim) { return (float)(((double)(splitmix64(s) >> 11) * 0x1p-53 * 2.0 - 1.0) * lim); };
    for (int i = 0; i < 320; ++i)
        p[kOW1 + i] = uni(std::sqrt(6.0 / 5.0));
    for (int i = 0; i < 4096; ++i)
        p[kOW2 + i] = uni(std::sqrt(6.0 / 64.0));
    for (int i = 0; i < 128; ++i)
        p[kOW3 + i] = uni(std::sqrt(6.0 / 64.0));
    const float norm[10] = {0, 0, 0, 0, 0, 1, 1, 1, 1, 1};
    const std::vector<float> zeros(kMlpParams, 0.f);
    slw_status st = hip_check(hipMemcpy(n->params, p.data(), kMlpParams * 4, hipMemcpyHostToDevice), "copy params");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(n->adam_m, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice), "zero moments");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(n->adam_v, zeros.data(), kMlpParams * 4, hipMemcpyHostToDevice), "zero moments");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(n->norm, norm, sizeof norm, hipMemcpyHostToDevice), "copy normalisation");
    if (st == SLW_OK)
        st = mlp_pack(n);
    if (st == SLW_OK)
        st = hip_check(hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (st != SLW_OK) {
        slw_mlp_free(n);
        return st;
    }
    *out = n;
    return SLW_OK;
}

slw_status slw_mlp_free(slw_mlp *n)
{
    if (!n)
        return SLW_OK;
    DeviceGuard gd(n->ctx->device);
    (void)hipStreamSynchronize(n->ctx->stream);
    void *ptrs[] = {n->params, n->adam_m, n->adam_v, n->grad, n->partial, n->norm, n->wpack, n->bias};
    for (void *p : ptrs)
        if (p)
            (void)hipFree(p);
    delete n;
    return SLW_OK;
}

slw_status slw_mlp_set_params(slw_mlp *n, const float *params_h)
{
    if (!n || !params_h)
        return set_error(SLW_E_ARG, "slw_mlp_set_params: null pointer");
    DeviceGuard gd(n->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(n->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(n->params, params_h, kMlpParams * 4, hipMemcpyHostToDevice), "copy params");
    if (st == SLW_OK)
        st = mlp_pack(n);
    return st;
}

slw_status slw_mlp_get_params(slw_mlp *n, float *params_h)
{
    if (!n || !params_h)
        return set_error(SLW_E_ARG, "slw_mlp_get_params: null pointer");
    DeviceGuard gd(n->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(n->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(params_h, n->params, kMlpParams * 4, hipMemcpyDeviceToHost), "copy params");
    return st;
}

slw_status slw_mlp_set_normalization(slw_mlp *n, const float *norm_h)
{
    if (!n || !norm_h)
        return set_error(SLW_E_ARG, "slw_mlp_set_normalization: null pointer");
    DeviceGuard gd(n->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(n->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(n->norm, norm_h, 10 * sizeof(float), hipMemcpyHostToDevice), "copy normalisation");
    return st;
}

slw_status slw_mlp_get_normalization(slw_mlp *n, float *norm_h)
{
    if (!n || !norm_h)
        return set_error(SLW_E_ARG, "slw_mlp_get_normalization: null pointer");
    DeviceGuard gd(n->ctx->device);
    slw_status st = hip_check(hipStreamSynchronize(n->ctx->stream), "hipStreamSynchronize");
    if (st == SLW_OK)
        st = hip_check(hipMemcpy(norm_h, n->norm, 10 * sizeof(float), hipMemcpyDeviceToHost), "copy normalisation");
    return st;
}

slw_status slw_mlp_fit_normalization(slw_mlp *n, const float *X, int64_t m)
{
    if (!n || m < 1 || !X)
        return set_error(SLW_E_ARG, "slw_mlp_fit_normalization: null pointer or no samples");
    DeviceGuard gd(n->ctx->device);
    // the partial sums live in the gradient partials' workspace (idle here)
    double *part = (double *)n->partial;
    static_assert((size_t)kNormParts * 10 * sizeof(double) <= (size_t)kMlpPartials * kPartialStride * sizeof(float),
                  "normalisation partials fit the gradient workspace");
    hipLaunchKernelGGL(k_fit_norm_partial, dim3(kNormParts), dim3(kBlock), 0, n->ctx->stream, X, m, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return hip_check(e, "slw_mlp_fit_normalization");
    hipLaunchKernelGGL(k_fit_norm_final, dim3(1), dim3(64), 0, n->ctx->stream, part, kNormParts, m, n->norm);
    return hip_check(hipGetLastError(), "slw_mlp_fit_normalization");
}

slw_status slw_learned_gather(slw_mesh *mesh, const slw_field *field, double t_np1, double dt, int scheme,
                              const int32_t *dofs, int64_t m, float *X, float *Y)
{
    if (!mesh || !field_ok(field) || m < 0 || (m > 0 && (!dofs || !X || !Y)))
        return set_error(SLW_E_ARG, "slw_learned_gather: null pointer, bad field or negative size");
    if (m > ((int64_t)1 << 31) - 1)
        return set_error(SLW_E_ARG, "slw_learned_gather: at most 2^31-1 samples per call");
    if (scheme != SLW_EULER && scheme != SLW_RK2)
        return set_error(SLW_E_ARG, "unknown scheme");
    if (!mesh->m.chart_uv)
        return set_error(SLW_E_ARG, "slw_learned_gather: no chart (slw_chart_build)");
    DeviceGuard gd(mesh->ctx->device);
    return hip_check(
        launch_learned_gather(mesh->m, mesh->ctx->stream, to_dev(field), t_np1, dt, scheme, dofs, m, X, Y),
        "slw_learned_gather");
}

slw_status slw_mlp_grad(slw_mlp *n, const float *X, const float *Y, int64_t m, float *grad_h, float *loss_h)
{
    if (!n || m < 1 || !X || !Y)
        return set_error(SLW_E_ARG, "slw_mlp_grad: null pointer or no samples");
    DeviceGuard gd(n->ctx->device);
    slw_status st = gradient_pass(n, X, Y, m, 0, m, 1, 0, 1.0f / (float)m);
    if (st == SLW_OK && grad_h)
        st = hip_check(hipMemcpyAsync(grad_h, n->grad, kMlpParams * 4, hipMemcpyDeviceToHost, n->ctx->stream),
                       "copy gradient");
    if (st == SLW_OK)
        st = read_loss(n, loss_h);
    return st;
}

slw_status slw_mlp_train(slw_mlp *n, const float *X, const float *Y, int64_t m, int epochs, int64_t batch,
                         float lr, uint64_t seed, float *loss_h)
{
    if (!n || m < 1 || !X || !Y || epochs < 1 || batch < 1 || !(lr > 0.f))
        return set_error(SLW_E_ARG, "slw_mlp_train: bad arguments");
    DeviceGuard gd(n->ctx->device);
    uint64_t s = seed;
    slw_status st = SLW_OK;
    for (int ep = 0; ep < epochs && st == SLW_OK; ++ep) {
        // this epoch's order i -> (a i + c) mod m with gcd(a, m) = 1
        uint64_t a = 1;
        if (m > 1) {
            do {
                a = splitmix64(s) % (uint64_t)m;
            } while (a == 0 || std::gcd(a, (uint64_t)m) != 1);
        }
        const uint64_t c = splitmix64(s) % (uint64_t)m;
        for (int64_t first = 0; first < m && st == SLW_OK; first += batch) {
            const int64_t count = std::min<int64_t>(batch, m - first);
            st = gradient_pass(n, X, Y, m, first, count, a, c, 1.0f / (float)count);
            if (st != SLW_OK)
                break;
            n->adam_t += 1;
            const float c1 = (float)(1.0 - std::pow(0.9, (double)n->adam_t));
            const float c2 = (float)(1.0 - std::pow(0.999, (double)n->adam_t));
            hipLaunchKernelGGL(k_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, n->ctx->stream, n->params,
                               n->adam_m, n->adam_v, n->grad, kMlpParams, lr, 0.9f, 0.999f, 1e-8f, c1, c2);
            st = hip_check(hipGetLastError(), "adam");
        }
    }
    if (st == SLW_OK)
        st = mlp_pack(n);
    if (st == SLW_OK)
        st = read_loss(n, loss_h);  // last minibatch, before its update
    return st;
}

slw_status slw_mlp_forward(slw_mlp *n, const float *X, int64_t m, float *out)
{
    if (!n || m < 0 || (m > 0 && (!X || !out)))
        return set_error(SLW_E_ARG, "slw_mlp_forward: null pointer or negative size");
    if (m == 0)
        return SLW_OK;
    if (m > ((int64_t)1 << 31) - 1)
        return set_error(SLW_E_ARG, "slw_mlp_forward: at most 2^31-1 samples per call");
    DeviceGuard gd(n->ctx->device);
    const unsigned g = (unsigned)((m + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(kBlock), 0, n->ctx->stream, n->wpack, n->bias, n->norm, X, m,
                       (float2 *)out);
    return hip_check(hipGetLastError(), "slw_mlp_forward");
}

slw_status slw_mesh_attach_mlp(slw_mesh *mesh, slw_mlp *n)
{
    if (!mesh)
        return set_error(SLW_E_ARG, "slw_mesh_attach_mlp: null mesh");
    if (n && n->ctx != mesh->ctx)
        return set_error(SLW_E_ARG, "slw_mesh_attach_mlp: network from another context");
    if (n && !mesh->m.chart_table)
        return set_error(SLW_E_ARG, "slw_mesh_attach_mlp: no chart (slw_chart_build)");
    mesh->m.mlp = n;  // the chart allocated the start workspace
    return SLW_OK;
}

}  // extern "C"

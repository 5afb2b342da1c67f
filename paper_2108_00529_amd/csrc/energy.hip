// ForceAtlas2 energy and its gradient (the negative ForceAtlas2 force field with exact
// repulsion), for gradient-based layout:
//   E = sum_e a_e d_e^2 / 2 - kr sum_{i<j} m_i m_j ln d_ij + kg sum_i m_i |x_i|
// Pair terms are evaluated in FP32 on LDS-staged 256x256 tiles; per-block partial
// sums are combined in FP64 in a fixed order.  The gradient splits the j range over
// several blocks per i tile and sums the splits in order, so no FP atomics are used.
#include <algorithm>

#include "common.h"
#include "fa2_internal.h"
#include "fa2_math.h"

namespace bgv {

constexpr int kEnThreads = 256;

__device__ __forceinline__ double block_sum(double v) {
    __shared__ double ws[kEnThreads / kWave];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int q = 0; q < kEnThreads / kWave; ++q) r += ws[q];
    __syncthreads();
    return r;
}

// Upper-triangular tile pairs (I <= J): block b -> (I, J).
__device__ __forceinline__ void tri_index(int64_t b, int T, int &I, int &J) {
    // row I holds T - I tiles; find I by walking (T is small: <= 2^23/256)
    int64_t rem = b;
    int i = 0;
    // closed form start, then fix up
    double tt = (double)T + 0.5;
    double est = tt - sqrt(tt * tt - 2.0 * (double)b);
    i = (int)est;
    if (i < 0) i = 0;
    if (i > T - 1) i = T - 1;
    auto start = [&](int r) { return (int64_t)r * T - (int64_t)r * (r - 1) / 2; };
    while (i > 0 && start(i) > b) --i;
    while (i < T - 1 && start(i + 1) <= b) ++i;
    rem = b - start(i);
    I = i;
    J = i + (int)rem;
}

constexpr double kLn2 = 0.693147180559945309417232121458176568;

// m_j log2 |x_i - x_j|^2 (none for coincident bodies), with the hardware base-2
// logarithm (within one ulp); subnormal d^2 is scaled by 2^64 first, since the
// instruction takes normal inputs.  The caller scales by ln 2.
__device__ __forceinline__ float en_log_term(float2 xi, float4 p) {
    const float dx = xi.x - p.x, dy = xi.y - p.y;
    const float d2 = dx * dx + dy * dy;
    const bool sub = d2 < 1.17549435e-38f;
    const float l = __builtin_amdgcn_logf(sub ? d2 * 18446744073709551616.0f : d2) - (sub ? 64.0f : 0.0f);
    return d2 > 0.f ? p.z * l : 0.f;
}

// Block x takes tile pairs x, x + grid, ... (one pair per block up to kEnPairBlocks
// pairs, i.e. up to about 740k supernodes; a fixed assignment and order either way).
__global__ void __launch_bounds__(kEnThreads) k_energy_pairs(int32_t K, int T, int64_t ntri,
                                                              const float2 *__restrict__ pos,
                                                              const float *__restrict__ mass,
                                                              double *__restrict__ part) {
    __shared__ float4 tile[kEnThreads];
    double acc = 0.0;
    for (int64_t pb = blockIdx.x; pb < ntri; pb += gridDim.x) {  // uniform over the workgroup
    int I, J;
    tri_index(pb, T, I, J);
    const int32_t i = I * kEnThreads + threadIdx.x;
    const int32_t j0 = J * kEnThreads;
    if (pb != blockIdx.x) __syncthreads();  // the previous pair's reads of the tile are done
    if (j0 + (int)threadIdx.x < K) {
        const float2 p = pos[j0 + threadIdx.x];
        tile[threadIdx.x] = make_float4(p.x, p.y, mass[j0 + threadIdx.x], 0.f);
    }
    __syncthreads();
    if (i < K) {
        const float2 xi = pos[i];
        const int cnt = min(kEnThreads, K - j0);
        float s = 0.f;
        // s = sum of m_j log2(d^2) over the tile's j above i; scaled by ln 2 below
        if (J > I && cnt == kEnThreads) {  // every j of the tile is above i
            for (int q = 0; q < kEnThreads; q += 8) {
                float4 b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) b[u] = tile[q + u];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += en_log_term(xi, b[u]);
            }
        } else {
            for (int q = 0; q < cnt; ++q) {
                const float v = en_log_term(xi, tile[q]);
                s += j0 + q > i ? v : 0.f;
            }
        }
        acc += 0.5 * kLn2 * (double)mass[i] * (double)s;
    }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kEnThreads) k_energy_edges(int64_t E, const int2 *__restrict__ edges,
                                                              const float *__restrict__ attr_w,
                                                              const float2 *__restrict__ pos,
                                                              double *__restrict__ part) {
    double acc = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kEnThreads + threadIdx.x; e < E; e += (int64_t)gridDim.x * kEnThreads) {
        const int2 p = edges[e];
        const float2 a = pos[p.x], b = pos[p.y];
        const float dx = a.x - b.x, dy = a.y - b.y;
        const float w = attr_w ? attr_w[e] : 1.0f;
        acc += 0.5 * (double)w * (double)(dx * dx + dy * dy);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

__global__ void __launch_bounds__(kEnThreads) k_energy_grav(int32_t K, const float2 *__restrict__ pos,
                                                             const float *__restrict__ mass,
                                                             double *__restrict__ part) {
    double acc = 0.0;
    for (int32_t i = blockIdx.x * kEnThreads + threadIdx.x; i < K; i += gridDim.x * kEnThreads) {
        const float2 p = pos[i];
        acc += (double)mass[i] * (double)sqrtf(p.x * p.x + p.y * p.y);
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// Fixed-order combination: E = att - kr * rep + kg * grav.
__global__ void __launch_bounds__(kEnThreads) k_energy_final(const double *__restrict__ prep, int nrep,
                                                              const double *__restrict__ patt, int natt,
                                                              const double *__restrict__ pgrav, int ngrav, float kr,
                                                              float kg, double *__restrict__ out) {
    double r = 0.0, a = 0.0, g = 0.0;
    for (int q = threadIdx.x; q < nrep; q += kEnThreads) r += prep[q];
    for (int q = threadIdx.x; q < natt; q += kEnThreads) a += patt[q];
    for (int q = threadIdx.x; q < ngrav; q += kEnThreads) g += pgrav[q];
    r = block_sum(r);
    a = block_sum(a);
    g = block_sum(g);
    if (threadIdx.x == 0) *out = a - (double)kr * r + (double)kg * g;
}

// Partial repulsion sums of the i tile over j split `blockIdx.y`.
__global__ void __launch_bounds__(kEnThreads) k_grad_rep(int32_t K, int jtiles_per_split,
                                                          const float2 *__restrict__ pos,
                                                          const float *__restrict__ mass,
                                                          float2 *__restrict__ prep) {
    __shared__ float4 tile[kEnThreads];
    const int32_t i = blockIdx.x * kEnThreads + threadIdx.x;
    const float2 xi = i < K ? pos[i] : make_float2(0.f, 0.f);
    float fx = 0.f, fy = 0.f;
    const int jt0 = blockIdx.y * jtiles_per_split;
    for (int jt = jt0; jt < jt0 + jtiles_per_split; ++jt) {
        const int32_t j0 = jt * kEnThreads;
        if (j0 >= K) break;
        if (j0 + (int)threadIdx.x < K) {
            const float2 p = pos[j0 + threadIdx.x];
            tile[threadIdx.x] = make_float4(p.x, p.y, mass[j0 + threadIdx.x], 0.f);
        }
        __syncthreads();
        const int cnt = min(kEnThreads, K - j0);
        if (cnt == kEnThreads) {
fa2_rep_run(xi, tile, kEnThreads, fx, fy);
        } else {
            for (int q = 0; q < cnt; ++q) fa2_rep_term(xi, tile[q], fx, fy);
        }
        __syncthreads();
    }
    if (i < K) prep[(int64_t)blockIdx.y * K + i] = make_float2(fx, fy);
}

// grad_i = -g * (kr m_i sum_splits rep + attraction + gravity)
__global__ void __launch_bounds__(kEnThreads) k_grad_final(int32_t K, int nsplit, const float2 *__restrict__ prep,
                                                            const float2 *__restrict__ pos,
                                                            const float *__restrict__ mass,
                                                            const float2 *__restrict__ att,
                                                            const uint32_t *__restrict__ item_of, float kr, float kg,
                                                            const float *__restrict__ grad_out,
                                                            float2 *__restrict__ grad) {
    for (int32_t i = blockIdx.x * kEnThreads + threadIdx.x; i < K; i += gridDim.x * kEnThreads) {
        float rx = 0.f, ry = 0.f;
        for (int q = 0; q < nsplit; ++q) {
            const float2 v = prep[(int64_t)q * K + i];
            rx += v.x;
            ry += v.y;
        }
        const float2 xi = pos[i];
        const float mi = mass[i];
        float fx = kr * mi * rx, fy = kr * mi * ry;
        const float2 a = fa2_att_combine(att, item_of, i);
        fx += a.x;
        fy += a.y;
        const float r = sqrtf(xi.x * xi.x + xi.y * xi.y);
        if (r > 0.f) {
            const float g = kg * mi / r;
            fx -= g * xi.x;
            fy -= g * xi.y;
        }
        const float go = grad_out ? *grad_out : 1.0f;
        grad[i] = make_float2(-go * fx, -go * fy);
    }
}

struct EnWs {
    CsrWs csr;
    double *prep, *patt, *pgrav;
    float2 *gsplit, *att;
};

static int en_tiles(int32_t K) { return (K + kEnThreads - 1) / kEnThreads; }
static int64_t en_tri_pairs(int32_t K) {
    const int64_t T = en_tiles(K);
    return T * (T + 1) / 2;
}
// larger supergraphs share their tile pairs out over this grid (4M workgroups of 256:
// under the 2^32 work-items a launch may have)
constexpr int64_t kEnPairBlocks = (int64_t)1 << 22;
static int64_t en_tri_blocks(int32_t K) { return std::min(en_tri_pairs(K), kEnPairBlocks); }
static int en_edge_blocks(int64_t E) { return (int)grid_for(E, kEnThreads * 8, 2048); }
static int en_grav_blocks(int32_t K) { return (int)grid_for(K, kEnThreads * 8, 2048); }
static int en_splits(int32_t K) {
    const int T = en_tiles(K);
    int s = (2048 + T - 1) / T;
    if (s > T) s = T;
    if (s < 1) s = 1;
    return s;
}

static size_t en_layout(Carver &c, int32_t K, int64_t E, EnWs *w) {
    csr_layout(c, K, E, &w->csr, false);  // one evaluation per call: no column-blocked setup
    w->prep = c.take<double>((size_t)en_tri_blocks(K));
    w->patt = c.take<double>((size_t)en_edge_blocks(E));
    w->pgrav = c.take<double>((size_t)en_grav_blocks(K));
    w->gsplit = c.take<float2>((size_t)en_splits(K) * (size_t)K);
    w->att = c.take<float2>((size_t)w->csr.items_bound);
    return c.size();
}

static bool en_valid(int32_t K, int64_t E) { return K >= 1 && K <= (1 << 24) && E >= 0 && E <= INT32_MAX; }

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_fa2_energy_workspace(int32_t K, int64_t E) {
    if (!en_valid(K, E)) return 0;
    Carver c(nullptr);
    EnWs w;
    return en_layout(c, K, E, &w);
}

extern "C" bgv_status bgv_fa2_energy(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                     const float *mass, const float *pos, float kr, float kg, double *energy,
                                     void *ws, size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (!en_valid(K, E) || (E > 0 && !edges) || !pos || !energy) {
        set_error("bgv_fa2_energy: invalid arguments (K=%d E=%lld)", K, (long long)E);
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_fa2_energy_workspace(K, E)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (range_check_on()) BGV_TRY(check_edge_ids(K, E, edges, reinterpret_cast<int32_t *>(energy), s));
    Carver c(ws);
    EnWs w;
    en_layout(c, K, E, &w);
    const float *m = mass;
    if (!m) BGV_TRY(build_csr(K, E, edges, attr_w, nullptr, w.csr, s, &m));
    const float2 *x = reinterpret_cast<const float2 *>(pos);
    const int64_t ntri = en_tri_blocks(K);
    BGV_LAUNCH(k_energy_pairs, dim3((unsigned)ntri), dim3(kEnThreads), 0, s, K, en_tiles(K), en_tri_pairs(K), x, m,
               w.prep);
    const int ne = en_edge_blocks(E), ng = en_grav_blocks(K);
    BGV_LAUNCH(k_energy_edges, dim3(ne), dim3(kEnThreads), 0, s, E, reinterpret_cast<const int2 *>(edges),
                       attr_w, x, w.patt);
    BGV_LAUNCH(k_energy_grav, dim3(ng), dim3(kEnThreads), 0, s, K, x, m, w.pgrav);
    BGV_LAUNCH(k_energy_final, dim3(1), dim3(kEnThreads), 0, s, w.prep, (int)ntri, w.patt, ne, w.pgrav, ng,
                       kr, kg, energy);
    return BGV_OK;
}

extern "C" bgv_status bgv_fa2_grad(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                   const float *mass, const float *pos, float kr, float kg, const float *grad_out,
                                   float *grad, void *ws, size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (!en_valid(K, E) || (E > 0 && !edges) || !pos || !grad) {
        set_error("bgv_fa2_grad: invalid arguments (K=%d E=%lld)", K, (long long)E);
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_fa2_energy_workspace(K, E)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (range_check_on()) BGV_TRY(check_edge_ids(K, E, edges, reinterpret_cast<int32_t *>(grad), s));
    Carver c(ws);
    EnWs w;
    en_layout(c, K, E, &w);
    const float *m = nullptr;
    BGV_TRY(build_csr(K, E, edges, attr_w, mass, w.csr, s, &m));
    const float2 *x = reinterpret_cast<const float2 *>(pos);
    const int T = en_tiles(K), ns = en_splits(K);
    const int per = (T + ns - 1) / ns;
    BGV_LAUNCH(k_grad_rep, dim3(T, ns), dim3(kEnThreads), 0, s, K, per, x, m, w.gsplit);
    BGV_TRY(attraction(K, x, w.csr, w.att, s));
    BGV_LAUNCH(k_grad_final, dim3(grid_for(K, kEnThreads, 65536)), dim3(kEnThreads), 0, s, K, ns, w.gsplit, x, m,
               w.att, w.csr.item_of, kr, kg, grad_out, reinterpret_cast<float2 *>(grad));
    return BGV_OK;
}

// ForceAtlas2 layout (Section 3.1 / Algorithm 1; force and speed laws of the cited
// ForceAtlas2 publication) on gfx950.
//
// Setup: directed CSR of the undirected edge list (own LSD radix sort, so neighbour
// order and therefore every FP sum is deterministic).
// Per iteration:
//   exact:  k_force_exact   LDS-tiled all-pairs repulsion + CSR attraction + gravity,
//                           swing/traction, FP64 block partials of the two sums
//   BH:     k_bh_bbox -> k_bh_codes -> radix sort -> k_bh_gather -> FP64 prefix sums
//           -> k_bh_build (binary radix tree; centre of mass of a node = difference of
//           prefix sums over its body range, so no atomics) -> k_bh_force (traversal)
//   both:   k_update        global speed from the partials (every block reduces them in
//                           the same order), local speeds, displacement
// No floating-point atomics anywhere: results are identical run to run.
#include "common.h"
#include "fa2_internal.h"

namespace bgv {

constexpr int kFaThreads = 256;
constexpr int kStackDepth = 64;

// ------------------------------------------------------------------------ CSR ----
__global__ void k_csr_keys(const int2 *__restrict__ edges, int64_t E, int kb, uint64_t *__restrict__ keys,
                           uint32_t *__restrict__ vals) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        const int2 p = edges[e];
        keys[2 * e] = ((uint64_t)(uint32_t)p.x << kb) | (uint32_t)p.y;
        keys[2 * e + 1] = ((uint64_t)(uint32_t)p.y << kb) | (uint32_t)p.x;
        vals[2 * e] = (uint32_t)e;
        vals[2 * e + 1] = (uint32_t)e;
    }
}

__global__ void k_csr_fill(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t nent,
                           int kb, int32_t K, const float *__restrict__ attr_w, uint32_t *__restrict__ row,
                           int32_t *__restrict__ col, float *__restrict__ w) {
    const uint64_t mask = (1ull << kb) - 1ull;
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < nent; k += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t key = keys[k];
        const int64_t src = (int64_t)(key >> kb);
        col[k] = (int32_t)(key & mask);
        w[k] = attr_w ? attr_w[vals[k]] : 1.0f;
        const int64_t prev = k ? (int64_t)(keys[k - 1] >> kb) : -1;
        for (int64_t r = prev + 1; r <= src; ++r) row[r] = (uint32_t)k;
        if (k == nent - 1)
            for (int64_t r = src + 1; r <= K; ++r) row[r] = (uint32_t)nent;
    }
}

__global__ void k_csr_mass(const uint32_t *__restrict__ row, int32_t K, float *__restrict__ mass) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < K; i += (int64_t)gridDim.x * blockDim.x)
        mass[i] = (float)(row[i + 1] - row[i]) + 1.0f;
}

static int bits_for(int64_t K) {
    int kb = 1;
    while (kb < 31 && (1ll << kb) < K) ++kb;
    return kb;
}

size_t csr_layout(Carver &c, int32_t K, int64_t E, CsrWs *w) {
    const int64_t nent = 2 * E > 0 ? 2 * E : 1;
    w->row = c.take<uint32_t>((size_t)K + 1);
    w->col = c.take<int32_t>((size_t)nent);
    w->wt = c.take<float>((size_t)nent);
    w->mass = c.take<float>((size_t)K);
    w->keys = c.take<uint64_t>((size_t)nent);
    w->keys_alt = c.take<uint64_t>((size_t)nent);
    w->vals = c.take<uint32_t>((size_t)nent);
    w->vals_alt = c.take<uint32_t>((size_t)nent);
    w->sort_scratch = c.take<char>(radix_workspace(nent));
    return c.size();
}

bgv_status build_csr(int32_t K, int64_t E, const int32_t *edges, const float *attr_w, const float *mass_in,
                     CsrWs &w, hipStream_t s, const float **mass_out) {
    if (E == 0) {
        BGV_TRY(fill<uint32_t>(w.row, 0u, (int64_t)K + 1, s));
    } else {
        const int kb = bits_for(K);
        hipLaunchKernelGGL(k_csr_keys, dim3(grid_for(E, kFaThreads, 65536)), dim3(kFaThreads), 0, s,
                           reinterpret_cast<const int2 *>(edges), E, kb, w.keys, w.vals);
        BGV_CHECK_LAUNCH();
        uint64_t *sk;
        uint32_t *sv;
        BGV_TRY(radix_sort_u64(w.keys, w.keys_alt, w.vals, w.vals_alt, 2 * E, 2 * kb, &sk, &sv, w.sort_scratch, s));
        hipLaunchKernelGGL(k_csr_fill, dim3(grid_for(2 * E, kFaThreads, 65536)), dim3(kFaThreads), 0, s, sk, sv,
                           2 * E, kb, K, attr_w, w.row, w.col, w.wt);
        BGV_CHECK_LAUNCH();
    }
    if (mass_in) {
        *mass_out = mass_in;
    } else {
        hipLaunchKernelGGL(k_csr_mass, dim3(grid_for(K, kFaThreads, 65536)), dim3(kFaThreads), 0, s, w.row, K,
                           w.mass);
        BGV_CHECK_LAUNCH();
        *mass_out = w.mass;
    }
    return BGV_OK;
}

// --------------------------------------------------------------- reductions ------
// Deterministic block sum of a double2 (fixed shuffle pattern, fixed wave order).
__device__ __forceinline__ double2 block_sum2(double2 v) {
    __shared__ double2 ws[kFaThreads / kWave];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        v.x += __shfl_down(v.x, o, kWave);
        v.y += __shfl_down(v.y, o, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if (threadIdx.x == 0)
        for (int q = 0; q < (int)(blockDim.x / kWave); ++q) {
            r.x += ws[q].x;
            r.y += ws[q].y;
        }
    __syncthreads();
    return r;  // valid in thread 0
}

// Attraction along CSR row i, gravity, then the swing/traction terms of node i.
__device__ __forceinline__ float2 attract_gravity(int32_t i, float2 xi, float mi, float2 frep,
                                                  const uint32_t *__restrict__ row, const int32_t *__restrict__ col,
                                                  const float *__restrict__ wt, const float2 *__restrict__ pos,
                                                  float kg) {
    float ax = 0.f, ay = 0.f;
    const uint32_t r0 = row[i], r1 = row[i + 1];
    for (uint32_t k = r0; k < r1; ++k) {
        const float2 xj = pos[col[k]];
        const float a = wt[k];
        ax += a * (xj.x - xi.x);
        ay += a * (xj.y - xi.y);
    }
    float fx = frep.x + ax, fy = frep.y + ay;
    const float r = sqrtf(xi.x * xi.x + xi.y * xi.y);
    if (r > 0.f) {
        const float g = kg * mi / r;
        fx -= g * xi.x;
        fy -= g * xi.y;
    }
    return make_float2(fx, fy);
}

__device__ __forceinline__ double2 swing_traction(float2 F, float2 Fp, float mi) {
    const float sx = F.x - Fp.x, sy = F.y - Fp.y;
    const float tx = F.x + Fp.x, ty = F.y + Fp.y;
    const float sw = sqrtf(sx * sx + sy * sy);
    const float tr = 0.5f * sqrtf(tx * tx + ty * ty);
    return make_double2((double)mi * (double)sw, (double)mi * (double)tr);
}

// ------------------------------------------------------------------ exact ------
__global__ void __launch_bounds__(kFaThreads) k_force_exact(int32_t K, const float2 *__restrict__ pos,
                                                             const float *__restrict__ mass,
                                                             const uint32_t *__restrict__ row,
                                                             const int32_t *__restrict__ col,
                                                             const float *__restrict__ wt, float kr, float kg,
                                                             const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                                             double2 *__restrict__ part) {
    __shared__ float4 tile[kFaThreads];
    const int32_t i = blockIdx.x * kFaThreads + threadIdx.x;
    const bool live = i < K;
    const float2 xi = live ? pos[i] : make_float2(0.f, 0.f);
    const float mi = live ? mass[i] : 0.f;
    float fx = 0.f, fy = 0.f;
    for (int32_t t0 = 0; t0 < K; t0 += kFaThreads) {
        const int32_t j = t0 + threadIdx.x;
        if (j < K) {
            const float2 xj = pos[j];
            tile[threadIdx.x] = make_float4(xj.x, xj.y, mass[j], 0.f);
        }
        __syncthreads();
        const int cnt = min(kFaThreads, K - t0);
        for (int q = 0; q < cnt; ++q) {
            const float4 p = tile[q];
            const float dx = xi.x - p.x, dy = xi.y - p.y;
            const float d2 = dx * dx + dy * dy;
            if (d2 > 0.f) {
                const float f = p.z / d2;
                fx += f * dx;
                fy += f * dy;
            }
        }
        __syncthreads();
    }
    double2 st = make_double2(0.0, 0.0);
    if (live) {
        const float c = kr * mi;
        const float2 f = attract_gravity(i, xi, mi, make_float2(c * fx, c * fy), row, col, wt, pos, kg);
        F[i] = f;
        st = swing_traction(f, fprev[i], mi);
    }
    st = block_sum2(st);
    if (threadIdx.x == 0) part[blockIdx.x] = st;
}

// ----------------------------------------------------------------- update ------
__global__ void __launch_bounds__(kFaThreads) k_update(int32_t K, float2 *__restrict__ pos,
                                                        float2 *__restrict__ fprev, const float2 *__restrict__ F,
                                                        const double2 *__restrict__ part, int32_t nparts,
                                                        const float *__restrict__ speed_in,
                                                        float *__restrict__ speed_out, float tau, float ks,
                                                        float ksmax) {
    __shared__ float s_speed;
    double2 acc = make_double2(0.0, 0.0);
    for (int p = threadIdx.x; p < nparts; p += kFaThreads) {
        acc.x += part[p].x;
        acc.y += part[p].y;
    }
    acc = block_sum2(acc);
    if (threadIdx.x == 0) {
        const float sp = *speed_in;
        float s = sp;
        if (acc.x > 0.0) s = (float)fmin((double)tau * acc.y / acc.x, 1.5 * (double)sp);
        s_speed = s;
        if (blockIdx.x == 0) *speed_out = s;
    }
    __syncthreads();
    const float s = s_speed;
    for (int32_t i = blockIdx.x * kFaThreads + threadIdx.x; i < K; i += gridDim.x * kFaThreads) {
        const float2 f = F[i], fp = fprev[i];
        const float sx = f.x - fp.x, sy = f.y - fp.y;
        const float sw = sqrtf(sx * sx + sy * sy);
        float si = ks * s / (1.0f + s * sqrtf(sw));
        const float fn = sqrtf(f.x * f.x + f.y * f.y);
        if (fn > 0.f && si > ksmax / fn) si = ksmax / fn;
        float2 p = pos[i];
        p.x += si * f.x;
        p.y += si * f.y;
        pos[i] = p;
        fprev[i] = f;
    }
}

__global__ void k_copy_f32(const float *__restrict__ a, float *__restrict__ b) { *b = *a; }

// ------------------------------------------------------------------ Barnes-Hut --
constexpr int kBboxBlocks = 64;

__global__ void __launch_bounds__(kFaThreads) k_bh_bbox(int32_t K, const float2 *__restrict__ pos,
                                                         float4 *__restrict__ part) {
    float xmn = INFINITY, xmx = -INFINITY, ymn = INFINITY, ymx = -INFINITY;
    for (int32_t i = blockIdx.x * kFaThreads + threadIdx.x; i < K; i += gridDim.x * kFaThreads) {
        const float2 p = pos[i];
        xmn = fminf(xmn, p.x);
        xmx = fmaxf(xmx, p.x);
        ymn = fminf(ymn, p.y);
        ymx = fmaxf(ymx, p.y);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        xmn = fminf(xmn, __shfl_down(xmn, o, kWave));
        xmx = fmaxf(xmx, __shfl_down(xmx, o, kWave));
        ymn = fminf(ymn, __shfl_down(ymn, o, kWave));
        ymx = fmaxf(ymx, __shfl_down(ymx, o, kWave));
    }
    __shared__ float4 ws[kFaThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = make_float4(xmn, xmx, ymn, ymx);
    __syncthreads();
    if (threadIdx.x == 0) {
        float4 r = ws[0];
        for (int q = 1; q < kFaThreads / kWave; ++q) {
            r.x = fminf(r.x, ws[q].x);
            r.y = fmaxf(r.y, ws[q].y);
            r.z = fminf(r.z, ws[q].z);
            r.w = fmaxf(r.w, ws[q].w);
        }
        part[blockIdx.x] = r;
    }
}

__device__ __forceinline__ uint32_t spread16(uint32_t v) {
    v &= 0xffffu;
    v = (v | (v << 8)) & 0x00ff00ffu;
    v = (v | (v << 4)) & 0x0f0f0f0fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

// Quantise on the 2^16 grid over the bounding square and Morton-encode (x even bits).
__global__ void __launch_bounds__(kFaThreads) k_bh_codes(int32_t K, const float2 *__restrict__ pos,
                                                          const float4 *__restrict__ part, int nparts,
                                                          uint64_t *__restrict__ keys, uint32_t *__restrict__ vals,
                                                          float *__restrict__ s0_out) {
    __shared__ float4 bb;
    if (threadIdx.x == 0) {
        float4 r = part[0];
        for (int q = 1; q < nparts; ++q) {
            r.x = fminf(r.x, part[q].x);
            r.y = fmaxf(r.y, part[q].y);
            r.z = fminf(r.z, part[q].z);
            r.w = fmaxf(r.w, part[q].w);
        }
        bb = r;
    }
    __syncthreads();
    const float xmin = bb.x, ymin = bb.z;
    const float ex = bb.y - bb.x, ey = bb.w - bb.z;
    float s0 = ex > ey ? ex : ey;
    if (!(s0 > 0.f)) s0 = 1.0f;
    if (blockIdx.x == 0 && threadIdx.x == 0) *s0_out = s0;
    for (int32_t i = blockIdx.x * kFaThreads + threadIdx.x; i < K; i += gridDim.x * kFaThreads) {
        const float2 p = pos[i];
        const float tx = __fdiv_rn(__fsub_rn(p.x, xmin), s0);
        const float ty = __fdiv_rn(__fsub_rn(p.y, ymin), s0);
        int32_t qx = (int32_t)__fmul_rn(tx, 65536.0f);
        int32_t qy = (int32_t)__fmul_rn(ty, 65536.0f);
        qx = qx > 65535 ? 65535 : qx;
        qy = qy > 65535 ? 65535 : qy;
        keys[i] = (uint64_t)(spread16((uint32_t)qx) | (spread16((uint32_t)qy) << 1));
        vals[i] = (uint32_t)i;
    }
}

// Bodies in Morton order: positions, masses, and FP64 mass moments for the prefix sums.
__global__ void k_bh_gather(int32_t K, const float2 *__restrict__ pos, const float *__restrict__ mass,
                            const uint64_t *__restrict__ skeys, const uint32_t *__restrict__ order,
                            float4 *__restrict__ body, uint32_t *__restrict__ code, double *__restrict__ dm,
                            double *__restrict__ dmx, double *__restrict__ dmy) {
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < K; k += gridDim.x * blockDim.x) {
        const uint32_t b = order[k];
        const float2 p = pos[b];
        const float m = mass[b];
        body[k] = make_float4(p.x, p.y, m, __int_as_float((int)b));
        code[k] = (uint32_t)skeys[k];
        dm[k] = (double)m;
        dmx[k] = (double)m * (double)p.x;
        dmy[k] = (double)m * (double)p.y;
    }
}

// Common-prefix length of sorted positions i and j; index bits break ties between
// equal codes (values >= 32 mean equal codes); -1 outside [0, K).
__device__ __forceinline__ int delta(const uint32_t *__restrict__ code, int32_t K, int32_t i, int32_t j) {
    if (j < 0 || j >= K) return -1;
    const uint32_t a = code[i], b = code[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz((uint32_t)i ^ (uint32_t)j);
}

// Internal node i of the binary radix tree over the sorted codes (Karras' parallel
// construction).  Children: >= 0 internal node, < 0 leaf ~child.  nodeA = (centre of
// mass, mass, size^2), size^2 < 0 for a node whose codes are all equal (a leaf cell).
__global__ void k_bh_build(int32_t K, const uint32_t *__restrict__ code, const double *__restrict__ PM,
                           const double *__restrict__ PX, const double *__restrict__ PY,
                           const float *__restrict__ s0p, float4 *__restrict__ nodeA, int4 *__restrict__ nodeB) {
    const float s0 = *s0p;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K - 1; i += gridDim.x * blockDim.x) {
        const int d = (delta(code, K, i, i + 1) - delta(code, K, i, i - 1)) >= 0 ? 1 : -1;
        const int dmin = delta(code, K, i, i - d);
        int lmax = 2;
        while (delta(code, K, i, i + lmax * d) > dmin) lmax <<= 1;
        int l = 0;
        for (int t = lmax >> 1; t >= 1; t >>= 1)
            if (delta(code, K, i, i + (l + t) * d) > dmin) l += t;
        const int j = i + l * d;
        const int dnode = delta(code, K, i, j);
        int sgap = 0;
        int t = l;
        do {
            t = (t + 1) >> 1;
            if (delta(code, K, i, i + (sgap + t) * d) > dnode) sgap += t;
        } while (t > 1);
        const int gamma = i + sgap * d + (d < 0 ? -1 : 0);
        const int first = min(i, j), last = max(i, j);
        const int left = (first == gamma) ? ~gamma : gamma;
        const int right = (last == gamma + 1) ? ~(gamma + 1) : gamma + 1;
        const double M = PM[last + 1] - PM[first];
        const double cx = (PX[last + 1] - PX[first]) / M;
        const double cy = (PY[last + 1] - PY[first]) / M;
        float size2;
        if (dnode >= 32) {
            size2 = -1.0f;
        } else {
            const int lev = min(dnode >> 1, 16);
            const float sz = s0 / (float)(1u << lev);
            size2 = sz * sz;
        }
        nodeA[i] = make_float4((float)cx, (float)cy, (float)M, size2);
        nodeB[i] = make_int4(left, right, first, last);
    }
}

__device__ __forceinline__ void add_pair(float2 xi, float4 bj, float &fx, float &fy) {
    const float dx = xi.x - bj.x, dy = xi.y - bj.y;
    const float d2 = dx * dx + dy * dy;
    if (d2 > 0.f) {
        const float f = bj.z / d2;
        fx += f * dx;
        fy += f * dy;
    }
}

// One thread per body in Morton order (neighbouring threads walk similar paths).
__global__ void __launch_bounds__(kFaThreads) k_bh_force(int32_t K, const float4 *__restrict__ body,
                                                          const float4 *__restrict__ nodeA,
                                                          const int4 *__restrict__ nodeB, float theta2,
                                                          const float2 *__restrict__ pos,
                                                          const uint32_t *__restrict__ row,
                                                          const int32_t *__restrict__ col,
                                                          const float *__restrict__ wt, float kr, float kg,
                                                          const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                                          double2 *__restrict__ part, int *__restrict__ overflow) {
    __shared__ int stack[kStackDepth][kFaThreads];
    const int32_t r = blockIdx.x * kFaThreads + threadIdx.x;
    double2 st = make_double2(0.0, 0.0);
    if (r < K) {
        const float4 me = body[r];
        const float2 xi = make_float2(me.x, me.y);
        const float mi = me.z;
        const int32_t b = __float_as_int(me.w);
        float fx = 0.f, fy = 0.f;
        int sp = 0;
        if (K > 1) stack[sp++][threadIdx.x] = 0;
        while (sp > 0) {
            const int node = stack[--sp][threadIdx.x];
            const float4 A = nodeA[node];
            const int4 Bn = nodeB[node];
            bool open;
            if (A.w < 0.f) {  // a cell of equal codes: direct sum
                for (int k = Bn.z; k <= Bn.w; ++k)
                    if (k != r) add_pair(xi, body[k], fx, fy);
                continue;
            } else if (r >= Bn.z && r <= Bn.w) {
                open = true;
            } else {
                const float dx = xi.x - A.x, dy = xi.y - A.y;
                const float d2 = dx * dx + dy * dy;
                if (d2 > 0.f && A.w < theta2 * d2) {
                    const float f = A.z / d2;
                    fx += f * dx;
                    fy += f * dy;
                    open = false;
                } else {
                    open = true;
                }
            }
            if (open) {
                // right first onto the stack so the left subtree is summed first
                if (Bn.y < 0) {
                    const int j = ~Bn.y;
                    if (j != r) add_pair(xi, body[j], fx, fy);
                } else if (sp < kStackDepth) {
                    stack[sp++][threadIdx.x] = Bn.y;
                } else {
                    *overflow = 1;
                }
                if (Bn.x < 0) {
                    const int j = ~Bn.x;
                    if (j != r) add_pair(xi, body[j], fx, fy);
                } else if (sp < kStackDepth) {
                    stack[sp++][threadIdx.x] = Bn.x;
                } else {
                    *overflow = 1;
                }
            }
        }
        const float c = kr * mi;
        const float2 f = attract_gravity(b, xi, mi, make_float2(c * fx, c * fy), row, col, wt, pos, kg);
        F[b] = f;
        st = swing_traction(f, fprev[b], mi);
    }
    st = block_sum2(st);
    if (threadIdx.x == 0) part[blockIdx.x] = st;
}

struct BhWs {
    float4 *bbox;
    float *s0;
    uint64_t *keys, *keys_alt;
    uint32_t *vals, *vals_alt;
    float4 *body;
    uint32_t *code;
    double *dm, *dmx, *dmy, *PM, *PX, *PY;
    float4 *nodeA;
    int4 *nodeB;
    int *overflow;
    void *sort_scratch, *scan_scratch;
};

struct FaWs {
    CsrWs csr;
    float2 *F;
    double2 *part;
    float *speed;  // [2] ping-pong
    BhWs bh;
};

static size_t fa_layout(Carver &c, int32_t K, int64_t E, const bgv_fa2_params *p, FaWs *w) {
    csr_layout(c, K, E, &w->csr);
    const int64_t nb = (K + kFaThreads - 1) / kFaThreads;
    w->F = c.take<float2>((size_t)K);
    w->part = c.take<double2>((size_t)nb);
    w->speed = c.take<float>(2);
    if (!p->exact) {
        BhWs &b = w->bh;
        b.bbox = c.take<float4>(kBboxBlocks);
        b.s0 = c.take<float>(1);
        b.keys = c.take<uint64_t>((size_t)K);
        b.keys_alt = c.take<uint64_t>((size_t)K);
        b.vals = c.take<uint32_t>((size_t)K);
        b.vals_alt = c.take<uint32_t>((size_t)K);
        b.body = c.take<float4>((size_t)K);
        b.code = c.take<uint32_t>((size_t)K);
        b.dm = c.take<double>((size_t)K);
        b.dmx = c.take<double>((size_t)K);
        b.dmy = c.take<double>((size_t)K);
        b.PM = c.take<double>((size_t)K + 1);
        b.PX = c.take<double>((size_t)K + 1);
        b.PY = c.take<double>((size_t)K + 1);
        b.nodeA = c.take<float4>((size_t)K);
        b.nodeB = c.take<int4>((size_t)K);
        b.overflow = c.take<int>(1);
        b.sort_scratch = c.take<char>(radix_workspace(K));
        b.scan_scratch = c.take<char>(scan_workspace(K));
    }
    return c.size();
}

static bool fa_valid(int32_t K, int64_t E, const bgv_fa2_params *p) {
    return p && K >= 1 && E >= 0 && E <= INT32_MAX && p->iters >= 0 && (p->exact == 0 || p->exact == 1) &&
           p->theta >= 0.f && p->tau > 0.f && p->ks >= 0.f && p->ksmax > 0.f;
}

// One Barnes-Hut repulsion + force evaluation into w.F / w.part.
static bgv_status bh_forces(int32_t K, const float2 *pos, const float *mass, const CsrWs &csr, float theta, float kr,
                            float kg, const float2 *fprev, FaWs &w, hipStream_t s) {
    BhWs &b = w.bh;
    const unsigned nb = (unsigned)((K + kFaThreads - 1) / kFaThreads);
    const int nbb = (int)grid_for(K, kFaThreads, kBboxBlocks);
    hipLaunchKernelGGL(k_bh_bbox, dim3(nbb), dim3(kFaThreads), 0, s, K, pos, b.bbox);
    BGV_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bh_codes, dim3(grid_for(K, kFaThreads, 4096)), dim3(kFaThreads), 0, s, K, pos, b.bbox, nbb,
                       b.keys, b.vals, b.s0);
    BGV_CHECK_LAUNCH();
    uint64_t *sk;
    uint32_t *sv;
    BGV_TRY(radix_sort_u64(b.keys, b.keys_alt, b.vals, b.vals_alt, K, 32, &sk, &sv, b.sort_scratch, s));
    hipLaunchKernelGGL(k_bh_gather, dim3(nb), dim3(kFaThreads), 0, s, K, pos, mass, sk, sv, b.body, b.code, b.dm,
                       b.dmx, b.dmy);
    BGV_CHECK_LAUNCH();
    BGV_TRY(exclusive_scan<double>(b.dm, b.PM, K, b.PM + K, b.scan_scratch, s));
    BGV_TRY(exclusive_scan<double>(b.dmx, b.PX, K, b.PX + K, b.scan_scratch, s));
    BGV_TRY(exclusive_scan<double>(b.dmy, b.PY, K, b.PY + K, b.scan_scratch, s));
    if (K > 1) {
        hipLaunchKernelGGL(k_bh_build, dim3(grid_for(K - 1, kFaThreads, 65536)), dim3(kFaThreads), 0, s, K, b.code,
                           b.PM, b.PX, b.PY, b.s0, b.nodeA, b.nodeB);
        BGV_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_bh_force, dim3(nb), dim3(kFaThreads), 0, s, K, b.body, b.nodeA, b.nodeB, theta * theta, pos,
                       csr.row, csr.col, csr.wt, kr, kg, fprev, w.F, w.part, b.overflow);
    BGV_CHECK_LAUNCH();
    return BGV_OK;
}

}  // namespace bgv

using namespace bgv;

extern "C" size_t bgv_fa2_workspace(int32_t K, int64_t E, const bgv_fa2_params *p) {
    if (!fa_valid(K, E, p)) return 0;
    Carver c(nullptr);
    FaWs w;
    return fa_layout(c, K, E, p, &w);
}

extern "C" bgv_status bgv_fa2_layout(int32_t K, int64_t E, const int32_t *edges, const float *attr_w,
                                     const float *mass, float *pos, float *fprev, float *speed,
                                     const bgv_fa2_params *p, void *ws, size_t ws_bytes, bgv_stream_t stream) {
    clear_error();
    if (!fa_valid(K, E, p)) {
        set_error("bgv_fa2_layout: invalid arguments (K=%d E=%lld)", K, (long long)E);
        return BGV_E_INVALID;
    }
    if ((E > 0 && !edges) || !pos || !fprev || !speed) {
        set_error("bgv_fa2_layout: null pointer");
        return BGV_E_INVALID;
    }
    BGV_TRY(check_ws(ws, ws_bytes, bgv_fa2_workspace(K, E, p)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Carver c(ws);
    FaWs w;
    fa_layout(c, K, E, p, &w);
    const float *m = nullptr;
    BGV_TRY(build_csr(K, E, edges, attr_w, mass, w.csr, s, &m));
    if (!p->exact) BGV_TRY(fill<int>(w.bh.overflow, 0, 1, s));

    float2 *x = reinterpret_cast<float2 *>(pos);
    float2 *fp = reinterpret_cast<float2 *>(fprev);
    const int32_t nb = (K + kFaThreads - 1) / kFaThreads;
    hipLaunchKernelGGL(k_copy_f32, dim3(1), dim3(1), 0, s, speed, w.speed);
    BGV_CHECK_LAUNCH();
    for (int32_t it = 0; it < p->iters; ++it) {
        if (p->exact) {
            hipLaunchKernelGGL(k_force_exact, dim3(nb), dim3(kFaThreads), 0, s, K, x, m, w.csr.row, w.csr.col,
                               w.csr.wt, p->kr, p->kg, fp, w.F, w.part);
            BGV_CHECK_LAUNCH();
        } else {
            BGV_TRY(bh_forces(K, x, m, w.csr, p->theta, p->kr, p->kg, fp, w, s));
        }
        hipLaunchKernelGGL(k_update, dim3(nb), dim3(kFaThreads), 0, s, K, x, fp, w.F, w.part, nb,
                           w.speed + (it & 1), w.speed + ((it + 1) & 1), p->tau, p->ks, p->ksmax);
        BGV_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(k_copy_f32, dim3(1), dim3(1), 0, s, w.speed + (p->iters & 1), speed);
    BGV_CHECK_LAUNCH();
    return BGV_OK;
}

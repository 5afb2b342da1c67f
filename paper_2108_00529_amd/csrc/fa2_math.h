// ForceAtlas2 per-pair and per-node arithmetic shared by the plain and batched layout
// kernels, so that both evaluate every force and speed with the same operation
// sequence (Section 3.1 / Algorithm 1, in the force and speed laws of the cited
// ForceAtlas2 publication).
#pragma once
#include "common.h"

namespace bgv {

// Repulsion from one body p = (x, y, mass): (x_i - x_j) * m_j / |x_i - x_j|^2, none if
// coincident.  The caller scales the sum by kr * m_i.  Branch-free so that unrolled
// loops keep several LDS reads in flight; 1/d^2 is the hardware reciprocal (within one
// ulp), the quotient's rounding being far below the layout's tolerance.
__device__ __forceinline__ void fa2_rep_term(float2 xi, float4 p, float &fx, float &fy) {
    const float dx = xi.x - p.x, dy = xi.y - p.y;
    const float d2 = dx * dx + dy * dy;
    const float f = d2 > 0.f ? p.z * __builtin_amdgcn_rcpf(d2) : 0.f;
    fx += f * dx;
    fy += f * dy;
}

// fa2_rep_term over n consecutive LDS bodies in ascending order, n a multiple of 8: each
// group of eight is read before any of it is used, so the reads overlap.
__device__ __forceinline__ void fa2_rep_run(float2 xi, const float4 *tile, int n, float &fx, float &fy) {
    for (int q = 0; q < n; q += 8) {
        float4 b[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) b[u] = tile[q + u];
#pragma unroll
        for (int u = 0; u < 8; ++u) fa2_rep_term(xi, b[u], fx, fy);
    }
}

// Exact repulsion on body i is summed over j in consecutive segments of kRepSegment
// bodies: each segment in ascending j starting from zero, then the segment sums in
// ascending order (the first one taken as is).  Segments let one body's sum be split
// over several workgroups while fixing the order of every addition, so any launch shape
// gives the same bits.  A multiple of the 256-body LDS tiles; short enough that a
// supergraph of a few thousand nodes spreads over many workgroups.
constexpr int32_t kRepSegment = 512;

__host__ __device__ __forceinline__ int32_t fa2_rep_segments(int32_t K) {
    return (K + kRepSegment - 1) / kRepSegment;
}

// CSR entries: (neighbour, weight bits) when edges are weighted, the bare neighbour id
// (32 or 16 bits) when every weight is 1.  Adding w * d with w = 1 rounds exactly like
// adding d (fused or not), so all three give the same bits for unit weights.
__device__ __forceinline__ int32_t fa2_entry_id(int2 e) { return e.x; }
__device__ __forceinline__ int32_t fa2_entry_id(uint32_t e) { return (int32_t)e; }
__device__ __forceinline__ int32_t fa2_entry_id(uint16_t e) { return (int32_t)e; }

__device__ __forceinline__ void fa2_entry_add(int2 e, float2 xj, float2 xi, float &ax, float &ay) {
    const float w = __int_as_float(e.y);
    ax += w * (xj.x - xi.x);
    ay += w * (xj.y - xi.y);
}
template <typename E>
__device__ __forceinline__ void fa2_entry_add(E, float2 xj, float2 xi, float &ax, float &ay) {
    ax += xj.x - xi.x;
    ay += xj.y - xi.y;
}

// Attraction over the CSR entries [b0, b1) of one block (at most kAttBlock entries), by
// one wavefront: lane l takes entries b0 + l, b0 + l + 64, ... in order (four loads in
// flight), then a fixed butterfly combines the lanes; every lane returns the total.
constexpr uint32_t kAttBlock = 16 * kWave;

template <typename E>
__device__ __forceinline__ float2 fa2_block_attraction(const float2 *__restrict__ pos, const E *__restrict__ cw,
                                                       uint32_t b0, uint32_t b1, float2 xi, int lane) {
    float ax = 0.f, ay = 0.f;
    uint32_t k = b0 + lane;
    // every lane adds its entries in ascending k; the unrolled loads only overlap
    for (; k + 7 * kWave < b1; k += 8 * kWave) {
        E e[8];
        float2 x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) e[u] = cw[k + u * kWave];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = pos[fa2_entry_id(e[u])];
#pragma unroll
        for (int u = 0; u < 8; ++u) fa2_entry_add(e[u], x[u], xi, ax, ay);
    }
    for (; k + 3 * kWave < b1; k += 4 * kWave) {
        const E e0 = cw[k], e1 = cw[k + kWave], e2 = cw[k + 2 * kWave], e3 = cw[k + 3 * kWave];
        const float2 x0 = pos[fa2_entry_id(e0)], x1 = pos[fa2_entry_id(e1)], x2 = pos[fa2_entry_id(e2)],
                     x3 = pos[fa2_entry_id(e3)];
        fa2_entry_add(e0, x0, xi, ax, ay);
        fa2_entry_add(e1, x1, xi, ax, ay);
        fa2_entry_add(e2, x2, xi, ax, ay);
        fa2_entry_add(e3, x3, xi, ax, ay);
    }
    for (; k < b1; k += kWave) {
        const E e = cw[k];
        fa2_entry_add(e, pos[fa2_entry_id(e)], xi, ax, ay);
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        ax += __shfl_xor(ax, o, kWave);
        ay += __shfl_xor(ay, o, kWave);
    }
    return make_float2(ax, ay);
}

// Attraction on node i = sum over its CSR entries [r0, r1) of w * (x_j - x_i): the row
// is cut into blocks of kAttBlock entries, each summed as above, and the block sums are
// added in order (the first taken as is).  A row of up to kAttBlock entries is a single
// block.  The blocks of a long (hub) row can then be summed by different wavefronts and
// combined afterwards with the same additions (fa2_att_combine).
template <typename E>
__device__ __forceinline__ float2 fa2_row_attraction(const float2 *__restrict__ pos, const E *__restrict__ cw,
                                                     uint32_t r0, uint32_t r1, float2 xi, int lane) {
    float2 t = fa2_block_attraction(pos, cw, r0, r1 - r0 > kAttBlock ? r0 + kAttBlock : r1, xi, lane);
    for (uint32_t b = r0 + kAttBlock; b < r1; b += kAttBlock) {
        const float2 v = fa2_block_attraction(pos, cw, b, r1 - b > kAttBlock ? b + kAttBlock : r1, xi, lane);
        t.x += v.x;
        t.y += v.y;
    }
    return t;
}

// Node i's attraction from its block sums attb[item_of[i] .. item_of[i + 1]), added in
// block order exactly as fa2_row_attraction adds them.
__device__ __forceinline__ float2 fa2_att_combine(const float2 *__restrict__ attb, const uint32_t *__restrict__ item_of,
                                                  int32_t i) {
    const uint32_t a = item_of[i], b = item_of[i + 1];
    float2 t = attb[a];
    for (uint32_t q = a + 1; q < b; ++q) {
        const float2 v = attb[q];
        t.x += v.x;
        t.y += v.y;
    }
    return t;
}

// Fixed-pattern sum of one double2 per thread over a group of 256 threads (4
// wavefronts): shuffle-down within each wavefront, then the 4 wavefront sums in order.
// ws must hold blockDim/64 entries; the result is valid in the group's first thread.
// Contains a barrier: every thread of the workgroup must call it.
__device__ __forceinline__ double2 fa2_sum256(double2 v, double2 *ws) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        v.x += __shfl_down(v.x, o, kWave);
        v.y += __shfl_down(v.y, o, kWave);
    }
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    if (lane == 0) ws[w] = v;
    __syncthreads();
    double2 r = make_double2(0.0, 0.0);
    if ((threadIdx.x & 255) == 0)
        for (int q = 0; q < 4; ++q) {
            r.x += ws[w + q].x;
            r.y += ws[w + q].y;
        }
    __syncthreads();
    return r;
}

// Net force: repulsion kr*m_i*sum + attraction + gravity (-kg m_i x / |x|, none at 0).
__device__ __forceinline__ float2 fa2_net_force(float2 xi, float mi, float kr, float rx, float ry, float2 att,
                                                float kg) {
    const float c = kr * mi;
    float fx = c * rx + att.x, fy = c * ry + att.y;
    const float r = sqrtf(xi.x * xi.x + xi.y * xi.y);
    if (r > 0.f) {
        const float g = kg * mi / r;
        fx -= g * xi.x;
        fy -= g * xi.y;
    }
    return make_float2(fx, fy);
}

// (m_i * swing_i, m_i * traction_i) with swing = |F - F'|, traction = |F + F'| / 2.
__device__ __forceinline__ double2 fa2_swing_traction(float2 F, float2 Fp, float mi) {
    const float sx = F.x - Fp.x, sy = F.y - Fp.y;
    const float tx = F.x + Fp.x, ty = F.y + Fp.y;
    const float sw = sqrtf(sx * sx + sy * sy);
    const float tr = 0.5f * sqrtf(tx * tx + ty * ty);
    return make_double2((double)mi * (double)sw, (double)mi * (double)tr);
}

// Global speed from the swing and traction sums: min(tau T / S, 1.5 s), kept if S = 0.
__device__ __forceinline__ float fa2_global_speed(double S, double T, float sp, float tau) {
    float s = sp;
    if (S > 0.0) s = (float)fmin((double)tau * T / S, 1.5 * (double)sp);
    return s;
}

// Local speed ks s / (1 + s sqrt(swing)), capped so the step is at most ksmax; moves p.
__device__ __forceinline__ float2 fa2_move(float2 p, float2 f, float2 fp, float s, float ks, float ksmax) {
    const float sx = f.x - fp.x, sy = f.y - fp.y;
    const float sw = sqrtf(sx * sx + sy * sy);
    float si = ks * s / (1.0f + s * sqrtf(sw));
    const float fn = sqrtf(f.x * f.x + f.y * f.y);
    if (fn > 0.f && si > ksmax / fn) si = ksmax / fn;
    p.x += si * f.x;
    p.y += si * f.y;
    return p;
}

// ---- whole-tile bodies shared by the plain kernels and the batched big-graph path ----
// A tile is 256 consecutive nodes handled by one 256-thread workgroup.
constexpr int kFa2Tile = 256;

// Node i's attraction: its CSR block sums combined (item_of != null) or a final value.
__device__ __forceinline__ float2 fa2_att_value(const float2 *__restrict__ att, const uint32_t *__restrict__ item_of,
                                                int32_t i) {
    return item_of ? fa2_att_combine(att, item_of, i) : att[i];
}

// Exact repulsion of the nodes of tile bx over the bodies of j segment by (all of
// [0, K) when kSegmented is false), bodies staged through LDS 256 at a time.  With one
// segment the tile's forces are finished (attraction, gravity, swing, traction and the
// tile's FP64 partial sums into part[bx]); with several, the segment sums go to seg.
template <bool kSegmented>
__device__ __forceinline__ void fa2_exact_force_tile(int32_t bx, int32_t by, int32_t K, const float2 *__restrict__ pos,
                                                     const float *__restrict__ mass, const float2 *__restrict__ att,
                                                     const uint32_t *__restrict__ item_of, float kr, float kg,
                                                     const float2 *__restrict__ fprev, float2 *__restrict__ F,
                                                     double2 *__restrict__ part, float2 *__restrict__ seg) {
    __shared__ float4 tile[kFa2Tile];
    __shared__ double2 ws[kFa2Tile / kWave];
    const int32_t i = bx * kFa2Tile + threadIdx.x;
    const bool live = i < K;
    const float2 xi = live ? pos[i] : make_float2(0.f, 0.f);
    const int32_t jb = kSegmented ? by * kRepSegment : 0;
    const int32_t je = kSegmented ? min(K, jb + kRepSegment) : K;
    float fx = 0.f, fy = 0.f;
    for (int32_t t0 = jb; t0 < je; t0 += kFa2Tile) {
        const int32_t j = t0 + threadIdx.x;
        if (j < je) {
            const float2 xj = pos[j];
            tile[threadIdx.x] = make_float4(xj.x, xj.y, mass[j], 0.f);
        }
        __syncthreads();
        const int cnt = min(kFa2Tile, je - t0);
        if (cnt == kFa2Tile) {
            fa2_rep_run(xi, tile, kFa2Tile, fx, fy);
        } else {
            for (int q = 0; q < cnt; ++q) fa2_rep_term(xi, tile[q], fx, fy);
        }
        __syncthreads();
    }
    if (kSegmented) {
        if (live) seg[(int64_t)by * K + i] = make_float2(fx, fy);
        return;
    }
    double2 st = make_double2(0.0, 0.0);
    if (live) {
        const float2 f = fa2_net_force(xi, mass[i], kr, fx, fy, fa2_att_value(att, item_of, i), kg);
        F[i] = f;
        st = fa2_swing_traction(f, fprev[i], mass[i]);
    }
    st = fa2_sum256(st, ws);
    if (threadIdx.x == 0) part[bx] = st;
}

// Segment sums of the nodes of tile bx added in ascending segment order, then the rest
// of the force as in fa2_exact_force_tile.
__device__ __forceinline__ void fa2_combine_tile(int32_t bx, int32_t K, int32_t nseg, const float2 *__restrict__ seg,
                                                 const float2 *__restrict__ pos, const float *__restrict__ mass,
                                                 const float2 *__restrict__ att, const uint32_t *__restrict__ item_of,
                                                 float kr, float kg, const float2 *__restrict__ fprev,
                                                 float2 *__restrict__ F, double2 *__restrict__ part) {
    __shared__ double2 ws[kFa2Tile / kWave];
    const int32_t i = bx * kFa2Tile + threadIdx.x;
    double2 st = make_double2(0.0, 0.0);
    if (i < K) {
        float2 r = seg[i];
        for (int32_t q = 1; q < nseg; ++q) {
            const float2 v = seg[(int64_t)q * K + i];
            r.x += v.x;
            r.y += v.y;
        }
        const float f_mi = mass[i];
        const float2 f = fa2_net_force(pos[i], f_mi, kr, r.x, r.y, fa2_att_value(att, item_of, i), kg);
        F[i] = f;
        st = fa2_swing_traction(f, fprev[i], f_mi);
    }
    st = fa2_sum256(st, ws);
    if (threadIdx.x == 0) part[bx] = st;
}

// Global speed from part[0, nparts) (every tile reduces them in the same order; tile 0
// stores it), then local speeds and displacement of the nodes bx*256 + t + q*stride.
// Returns the thread's bounding box (xmin, xmax, ymin, ymax) of the moved positions.
// The global speed from part[0, nparts) by one 256-thread block (fixed order); every
// thread gets it.
__device__ __forceinline__ float fa2_speed_of_parts(const double2 *__restrict__ part, int32_t nparts,
                                                    const float *__restrict__ speed_in, float tau) {
    __shared__ float s_speed;
    __shared__ double2 ws[kFa2Tile / kWave];
    double2 acc = make_double2(0.0, 0.0);
    for (int p = threadIdx.x; p < nparts; p += kFa2Tile) {
        acc.x += part[p].x;
        acc.y += part[p].y;
    }
    acc = fa2_sum256(acc, ws);
    if (threadIdx.x == 0) s_speed = fa2_global_speed(acc.x, acc.y, *speed_in, tau);
    __syncthreads();
    return s_speed;
}

// Local speeds and displacement, at global speed s, of the nodes bx*256 + t + q*stride;
// returns the thread's bounding box (xmin, xmax, ymin, ymax) of the moved positions.
__device__ __forceinline__ float4 fa2_move_tile(int32_t bx, int32_t stride, int32_t K, float2 *__restrict__ pos,
                                                float2 *__restrict__ fprev, const float2 *__restrict__ F, float s,
                                                float ks, float ksmax) {
    const float inf = __builtin_huge_valf();
    float4 bb = make_float4(inf, -inf, inf, -inf);
    for (int32_t i = bx * kFa2Tile + threadIdx.x; i < K; i += stride * kFa2Tile) {
        const float2 f = F[i];
        const float2 p = fa2_move(pos[i], f, fprev[i], s, ks, ksmax);
        pos[i] = p;
        fprev[i] = f;
        bb = make_float4(fminf(bb.x, p.x), fmaxf(bb.y, p.x), fminf(bb.z, p.y), fmaxf(bb.w, p.y));
    }
    return bb;
}

__device__ __forceinline__ float4 fa2_update_tile(int32_t bx, int32_t stride, int32_t K, float2 *__restrict__ pos,
                                                  float2 *__restrict__ fprev, const float2 *__restrict__ F,
                                                  const double2 *__restrict__ part, int32_t nparts,
                                                  const float *__restrict__ speed_in, float *__restrict__ speed_out,
                                                  float tau, float ks, float ksmax) {
    const float s = fa2_speed_of_parts(part, nparts, speed_in, tau);
    if (bx == 0 && threadIdx.x == 0) *speed_out = s;
    return fa2_move_tile(bx, stride, K, pos, fprev, F, s, ks, ksmax);
}

}  // namespace bgv

// Level 2 summaries and position statistics of L1 halos (end of Sec. 2.2.2,
// Table 1), after the L2 pass has run with the L1 halos as groups.
//
//   centres   one workgroup per L1 halo: the centre of mass of its members
//             (x_com) and of the members of its first L2 halo (x_L2com), each
//             about a reference particle (the L1 / L2 nucleus): minimum-image
//             offsets rounded to multiples of 2^-32 and summed exactly in
//             64-bit integers, so the sums do not depend on the member order
//             or the reduction shape;
//   distances squared distance of every member from x_L2com (FP64, rounded to
//             float32), keyed (halo, distance) and radix sorted, so every halo's
//             distances come out sorted in its own member range;
//   radial    r_XX = the k-th smallest distance with k = ceil(XX N / 100);
//             vcirc: k members lie within the k-th distance r_k, the circular
//             velocity sqrt(m_p k / r_k) (G = 1) is largest at the first k
//             maximising k^2 / r_k^2 (members at r = 0 skipped);
//   members   the L1 members grouped by halo (ascending id, ascending index).
#include "hf_internal.h"

namespace hf {

namespace {

inline dim3 grid(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

constexpr int kNumPct = 9;
__constant__ int kPct[kNumPct] = {10, 25, 33, 50, 67, 75, 90, 95, 98};
constexpr double kFix = 4294967296.0;  // 2^32

__device__ __forceinline__ double fold(double d, const Geo &g) {
    return d > g.half ? d - g.L : (d < -g.half ? d + g.L : d);
}

// Block-wide sum of a 64-bit integer (256 threads); the result is returned to
// every thread.
__device__ __forceinline__ long long block_sum_i64(long long v, long long *s) {
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < kBlock / 64; w++) t += s[w];
    return t;
}

__global__ __launch_bounds__(kBlock) void k_stats_centres(int G, Geo g, double particle_mass,
                                                          const float *__restrict__ pos,
                                                          const int32_t *__restrict__ g_start,
                                                          const int32_t *__restrict__ g_size,
                                                          const int32_t *__restrict__ g_label,
                                                          const int32_t *__restrict__ mem,
                                                          const float4 *__restrict__ spos,
                                                          const int32_t *__restrict__ owner,
                                                          const uint32_t *__restrict__ gcoff,
                                                          const int32_t *__restrict__ g_nh,
                                                          const int32_t *__restrict__ h_nuc,
                                                          const uint32_t *__restrict__ h_count,
                                                          double *__restrict__ gcom,
                                                          int32_t *__restrict__ ordk,
                                                          hf_halo_summary *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ long long s_red[kBlock / 64];
    const int gi = blockIdx.x;
    const int64_t start = g_start[gi], m = g_size[gi];
    const int key = g_label[gi] - 1;
    const int nh = g_nh[gi];
    const int first = nh > 0 ? (int)gcoff[gi] : -1;
    const double r1[3] = {(double)pos[3 * (int64_t)key], (double)pos[3 * (int64_t)key + 1],
                          (double)pos[3 * (int64_t)key + 2]};
    double r2[3] = {r1[0], r1[1], r1[2]};
    if (first >= 0) {
        const float4 q = spos[h_nuc[first]];
        r2[0] = q.x;
        r2[1] = q.y;
        r2[2] = q.z;
    }
    long long a1[3] = {0, 0, 0}, a2[3] = {0, 0, 0}, c2 = 0;
    for (int64_t t = threadIdx.x; t < m; t += kBlock) {
        const int slot = mem[start + t];
        const float4 q = spos[slot];
        const double x[3] = {q.x, q.y, q.z};
        for (int a = 0; a < 3; a++) a1[a] += __double2ll_rn(fold(x[a] - r1[a], g) * kFix);
        if (first >= 0 && owner[slot] == first) {
            for (int a = 0; a < 3; a++) a2[a] += __double2ll_rn(fold(x[a] - r2[a], g) * kFix);
            c2++;
        }
    }
    long long S1[3], S2[3];
    for (int a = 0; a < 3; a++) {
        S1[a] = block_sum_i64(a1[a], s_red);
        S2[a] = block_sum_i64(a2[a], s_red);
    }
    const long long C2 = block_sum_i64(c2, s_red);
    if (threadIdx.x != 0) return;
    double com1[3], com2[3];
    for (int a = 0; a < 3; a++) {
        double c = (double)S1[a];
        c = c / (double)m;
        c = c * (1.0 / kFix);
        double x = r1[a] + c;
        com1[a] = x < 0.0 ? x + g.L : (x >= g.L ? x - g.L : x);
        if (first >= 0) {
            double e = (double)S2[a];
            e = e / (double)C2;
            e = e * (1.0 / kFix);
            double y = r2[a] + e;
            com2[a] = y < 0.0 ? y + g.L : (y >= g.L ? y - g.L : y);
        } else {
            com2[a] = com1[a];
        }
        gcom[6 * (int64_t)gi + a] = com1[a];
        gcom[6 * (int64_t)gi + 3 + a] = com2[a];
    }
    ordk[key] = gi;
    hf_halo_summary st = {};
    st.id = key + 1;
    st.n = (int32_t)m;
    st.n_l2 = nh;
    st.l2max_nucleus = first >= 0 ? (int32_t)orig_of(spos[h_nuc[first]]) : -1;
    st.l2max_n = first >= 0 ? (int32_t)h_count[first] : 0;
    for (int a = 0; a < 3; a++) {
        st.x_com[a] = (float)com1[a];
        st.x_l2com[a] = (float)com2[a];
    }
    // the five largest L2 halos, by member count
    uint32_t top[5] = {0, 0, 0, 0, 0};
    for (int h = 0; h < nh; h++) {
        uint32_t v = h_count[first + h];
        for (int u = 0; u < 5; u++)
            if (v > top[u]) {
                const uint32_t t = top[u];
                top[u] = v;
                v = t;
            }
    }
    for (int u = 0; u < 5; u++) st.l2_mass[u] = (float)((double)top[u] * particle_mass);
    out[gi] = st;
}

// Sort key of every member (in member order): (halo, float32 squared distance
// from x_L2com); squared distances are >= 0, so their bits order like values.
__global__ __launch_bounds__(kBlock) void k_stats_keys(int64_t M, Geo g, const int32_t *__restrict__ mem,
                                                       const int32_t *__restrict__ gid_of,
                                                       const float4 *__restrict__ spos,
                                                       const double *__restrict__ gcom,
                                                       uint64_t *__restrict__ keys) {
#pragma clang fp contract(off)
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= M) return;
    const int slot = mem[t];
    const int gi = gid_of[slot];
    const float4 q = spos[slot];
    const double *c = gcom + 6 * (int64_t)gi + 3;
    const double dx = fold((double)q.x - c[0], g), dy = fold((double)q.y - c[1], g),
                 dz = fold((double)q.z - c[2], g);
    const float d2 = (float)((dx * dx + dy * dy) + dz * dz);
    keys[t] = ((uint64_t)(uint32_t)gi << 32) | (uint64_t)__float_as_uint(d2);
}

__device__ __forceinline__ float key_d2(uint64_t k) { return __uint_as_float((uint32_t)k); }

__global__ __launch_bounds__(kBlock) void k_stats_radial(int G, double particle_mass,
                                                         const int32_t *__restrict__ g_start,
                                                         const int32_t *__restrict__ g_size,
                                                         const uint64_t *__restrict__ keys,
                                                         hf_halo_summary *__restrict__ out) {
#pragma clang fp contract(off)
    __shared__ double s_v[kBlock / 64];
    __shared__ int64_t s_t[kBlock / 64];
    const int gi = blockIdx.x;
    const int64_t start = g_start[gi], m = g_size[gi];
    const uint64_t *k = keys + start;
    if (threadIdx.x < kNumPct) {
        const int64_t kk = ((int64_t)kPct[threadIdx.x] * m + 99) / 100;
        out[gi].r_pct[threadIdx.x] = (float)sqrt((double)key_d2(k[kk - 1]));
    }
    // first position maximising (t+1)^2 / d2_t over d2_t > 0
    double bv = -1.0;
    int64_t bt = -1;
    for (int64_t t = threadIdx.x; t < m; t += kBlock) {
        const float f = key_d2(k[t]);
        if (!(f > 0.0f)) continue;
        const double v = ((double)(t + 1) * (double)(t + 1)) / (double)f;
        if (v > bv) {
            bv = v;
            bt = t;
        }
    }
    for (int d = 32; d >= 1; d >>= 1) {
        const double ov = __shfl_xor(bv, d, 64);
        const int64_t ot = __shfl_xor(bt, d, 64);
        if (ov > bv || (ov == bv && ot >= 0 && (bt < 0 || ot < bt))) {
            bv = ov;
            bt = ot;
        }
    }
    if ((threadIdx.x & 63) == 0) {
        s_v[threadIdx.x >> 6] = bv;
        s_t[threadIdx.x >> 6] = bt;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int w = 1; w < kBlock / 64; w++)
        if (s_v[w] > bv || (s_v[w] == bv && s_t[w] >= 0 && (bt < 0 || s_t[w] < bt))) {
            bv = s_v[w];
            bt = s_t[w];
        }
    if (bt >= 0) {
        const double r = sqrt((double)key_d2(k[bt]));
        out[gi].vcirc_max = (float)sqrt((particle_mass * (double)(bt + 1)) / r);
        out[gi].rvcirc_max = (float)r;
    } else {
        out[gi].vcirc_max = 0.0f;
        out[gi].rvcirc_max = 0.0f;
    }
}

// Group-ordered listing: members in original order keyed (halo ordinal, index).
__global__ __launch_bounds__(kBlock) void k_members_flags(int64_t n, const int32_t *__restrict__ halo_id,
                                                          uint32_t *__restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = halo_id[i] > 0 ? 1u : 0u;
}

__global__ __launch_bounds__(kBlock) void k_members_keys(int64_t n, const int32_t *__restrict__ halo_id,
                                                         const int32_t *__restrict__ ordk,
                                                         const uint32_t *__restrict__ flag,
                                                         const uint32_t *__restrict__ at,
                                                         uint64_t *__restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !flag[i]) return;
    keys[at[i]] = ((uint64_t)(uint32_t)ordk[halo_id[i] - 1] << 32) | (uint64_t)i;
}

__global__ __launch_bounds__(kBlock) void k_members_out(int64_t M, int G, const uint64_t *__restrict__ keys,
                                                        const int32_t *__restrict__ g_start,
                                                        int32_t *__restrict__ members,
                                                        int32_t *__restrict__ group_start) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (members && t < M) members[t] = (int32_t)(uint32_t)keys[t];
    if (group_start && t <= G) group_start[t] = t < G ? g_start[t] : (int32_t)M;
}

int bit_width64(uint64_t x) {
    int b = 0;
    while (b < 64 && (x >> b)) b++;
    return b;
}

}  // namespace

void launch_halo_stats(int64_t n, int64_t G, int64_t M, const Geo &g, double particle_mass, const float *pos,
                       const int32_t *halo_id, Work &w, hf_halo_summary *out, int32_t *group_start,
                       int32_t *group_members, hipStream_t s) {
    if (G <= 0) return;
    hipLaunchKernelGGL(k_stats_centres, dim3((unsigned)G), dim3(kBlock), 0, s, (int)G, g, particle_mass, pos,
                       w.g_start, w.g_size, w.g_label, w.mem, w.spos, w.owner, w.gcoff, w.g_nh, w.h_nuc,
                       w.h_count, w.gcom, w.ordk, out);
    hipLaunchKernelGGL(k_stats_keys, grid(M), dim3(kBlock), 0, s, M, g, w.mem, w.gid_of, w.spos, w.gcom,
                       w.rkey[0]);
    const int gbits = bit_width64((uint64_t)(G - 1));
    const uint64_t *sorted = radix_sort_keys(w.rkey[0], w.rkey[1], M, 0, 32 + gbits, w, s);
    hipLaunchKernelGGL(k_stats_radial, dim3((unsigned)G), dim3(kBlock), 0, s, (int)G, particle_mass, w.g_start,
                       w.g_size, sorted, out);
    if (!group_start && !group_members) return;
    uint64_t *lk = nullptr;
    if (group_members) {
        hipLaunchKernelGGL(k_members_flags, grid(n), dim3(kBlock), 0, s, n, halo_id, w.f_chunk);
        scan_u32(w.f_chunk, w.s_chunk, n, w.scan_tmp, s);
        hipLaunchKernelGGL(k_members_keys, grid(n), dim3(kBlock), 0, s, n, halo_id, w.ordk, w.f_chunk, w.s_chunk,
                           w.rkey[0]);
        // the index bits are already in order: sort by the ordinal bits only
        lk = radix_sort_keys(w.rkey[0], w.rkey[1], M, 32, gbits > 0 ? gbits : 1, w, s);
    }
    hipLaunchKernelGGL(k_members_out, grid(M > G + 1 ? M : G + 1), dim3(kBlock), 0, s, M, (int)G, lk, w.g_start,
                       group_members, group_start);
}

}  // namespace hf

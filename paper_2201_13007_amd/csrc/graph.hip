// Graph construction for the search (the paper takes a prebuilt NSG graph, Sec. 2.2;
// this builds the fixed-width graph the kernels read): the medoid entry point, row
// pruning of exact candidate lists, and a connectivity repair.
//
// Every distance here is computed by one thread walking the dimensions in index order in
// double precision (separately rounded multiply and add) and rounded once to float, so
// each pruning and bridging decision is reproducible bit for bit.
#include "sa_internal.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace sa {
namespace {

__device__ float dist_seq(const float *a, const float *b, int d, int metric)
{
    double acc = 0.0;
    if (metric == SA_L2) {
        for (int i = 0; i < d; i += 4) {
            const float4 x = *reinterpret_cast<const float4 *>(a + i);
            const float4 y = *reinterpret_cast<const float4 *>(b + i);
            double t;
            t = (double)x.x - (double)y.x; acc += t * t;
            t = (double)x.y - (double)y.y; acc += t * t;
            t = (double)x.z - (double)y.z; acc += t * t;
            t = (double)x.w - (double)y.w; acc += t * t;
        }
        return (float)acc;
    }
    for (int i = 0; i < d; i += 4) {
        const float4 x = *reinterpret_cast<const float4 *>(a + i);
        const float4 y = *reinterpret_cast<const float4 *>(b + i);
        acc += (double)x.x * (double)y.x;
        acc += (double)x.y * (double)y.y;
        acc += (double)x.z * (double)y.z;
        acc += (double)x.w * (double)y.w;
    }
    return (float)(-acc);
}

// ---------------------------------------------------------------- medoid

constexpr int MED_CHUNK = 4096;

__global__ void colsum_partial(const float *base, int64_t n, int d, int64_t ld, double *part)
{
    const int64_t r0 = (int64_t)blockIdx.x * MED_CHUNK;
    const int64_t r1 = min(n, r0 + MED_CHUNK);
    for (int c = threadIdx.x; c < d; c += blockDim.x) {
        double s = 0.0;
        for (int64_t r = r0; r < r1; ++r) s += (double)base[r * ld + c];
        part[(int64_t)blockIdx.x * d + c] = s;
    }
}

__global__ void colsum_final(const double *part, int64_t nchunks, int d, int64_t n, double *mean)
{
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < d; c += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int64_t b = 0; b < nchunks; ++b) s += part[b * d + c];
        mean[c] = s / (double)n;
    }
}

__global__ void dist_to_mean(const float *base, int64_t n, int d, int64_t ld, const double *mean, double *bestd,
                             int64_t *besti)
{
    __shared__ double sd[256];
    __shared__ int64_t si[256];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc = INFINITY;
    int64_t id = INT64_MAX;
    if (r < n) {
        acc = 0.0;
        for (int c = 0; c < d; ++c) {
            double t = (double)base[r * ld + c] - mean[c];
            acc += t * t;
        }
        id = r;
    }
    sd[threadIdx.x] = acc;
    si[threadIdx.x] = id;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            double od = sd[threadIdx.x + s];
            int64_t oi = si[threadIdx.x + s];
            if (od < sd[threadIdx.x] || (od == sd[threadIdx.x] && oi < si[threadIdx.x])) {
                sd[threadIdx.x] = od;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bestd[blockIdx.x] = sd[0];
        besti[blockIdx.x] = si[0];
    }
}

// ---------------------------------------------------------------- pruning

__global__ void prune_kernel(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *cand,
                             int kc, int R, int mode, int32_t *adj)
{
    __shared__ int32_t kept_all[4][64];
    const int wv = threadIdx.x >> 6, lane = __lane_id();
    const int64_t p = (int64_t)blockIdx.x * 4 + wv;
    if (p >= n) return;
    int32_t *kept = kept_all[wv];
    int32_t c_mine = lane < kc ? cand[p * kc + lane] : -1;
    if (c_mine >= n) c_mine = -1;   // malformed candidates are ignored like padding
    int nk = 0;
    if (mode == 0) {
        const uint64_t m = __ballot(c_mine >= 0);
        const int pos = __popcll(m & ((1ull << lane) - 1ull));
        if (c_mine >= 0 && pos < R) kept[pos] = c_mine;
        nk = min(R, __popcll(m));
    } else {
        const float dpc_mine = c_mine >= 0 ? dist_seq(base + p * ld, base + (int64_t)c_mine * ld, d, metric) : 0.f;
        for (int j = 0; j < kc && nk < R; ++j) {
            const int32_t c = __shfl(c_mine, j, 64);
            if (c < 0) continue;
            const float dpc = __shfl(dpc_mine, j, 64);
            bool occl = false;
            if (lane < nk) {
                const int32_t s = kept[lane];
                occl = dist_seq(base + (int64_t)s * ld, base + (int64_t)c * ld, d, metric) < dpc;
            }
            if (__ballot(occl) == 0) {
                __builtin_amdgcn_wave_barrier();
                if (lane == 0) kept[nk] = c;
                __builtin_amdgcn_wave_barrier();
                ++nk;
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < R; j += 64) adj[p * R + j] = j < nk ? kept[j] : -1;
}

// ---------------------------------------------------------------- repair helpers

// For several vertices at once: results[j] = the smallest key (distance to us[j], id)
// over the marked vertices with a free slot (grid.y = j); results start as KEY_EMPTY
__global__ void nearest_marked_batch(const float *base, int64_t n, int d, int64_t ld, int metric, const uint8_t *mask,
                                     const int32_t *deg, int R, const int32_t *us, unsigned long long *results)
{
    __shared__ unsigned long long sk[256];
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t u = us[blockIdx.y];
    unsigned long long key = KEY_EMPTY;
    if (w < n && mask[w] && deg[w] < R) {
        float dd = dist_seq(base + w * ld, base + (int64_t)u * ld, d, metric);
        key = make_key(dd, (int32_t)w);
    }
    sk[threadIdx.x] = key;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s && sk[threadIdx.x + s] < sk[threadIdx.x]) sk[threadIdx.x] = sk[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0 && sk[0] != KEY_EMPTY) atomicMin(results + blockIdx.y, sk[0]);
}

__global__ void fill_u64_n(unsigned long long *p, int64_t cnt, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cnt) p[i] = v;
}

// distance of every edge p -> c, computed as d(c, p)
__global__ void edge_dists(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *adj, int R,
                           float *out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * R) return;
    const int64_t p = e / R;
    const int32_t c = adj[e];
    out[e] = (c >= 0 && c < n) ? dist_seq(base + (int64_t)c * ld, base + p * ld, d, metric) : 0.f;
}

// host-side distance with the same arithmetic as dist_seq
float host_dist(const float *a, const float *b, int d, int metric)
{
    double acc = 0.0;
    if (metric == SA_L2) {
        for (int i = 0; i < d; ++i) {
            double t = (double)a[i] - (double)b[i];
            acc += t * t;
        }
        return (float)acc;
    }
    for (int i = 0; i < d; ++i) acc += (double)a[i] * (double)b[i];
    return (float)(-acc);
}

bool key_less_host(float da, int32_t ia, float db, int32_t ib) { return da < db || (da == db && ia < ib); }

// medoid of a set of rows: mean summed in the listed order, then the nearest row
int32_t host_medoid(const float *X, int64_t ld, int d, const int32_t *members, int64_t cnt)
{
    std::vector<double> mean(d, 0.0);
    for (int64_t a = 0; a < cnt; ++a) {
        const float *x = X + (int64_t)members[a] * ld;
        for (int i = 0; i < d; ++i) mean[i] += (double)x[i];
    }
    for (int i = 0; i < d; ++i) mean[i] /= (double)cnt;
    int32_t best = -1;
    double bestd = INFINITY;
    for (int64_t a = 0; a < cnt; ++a) {
        const int32_t v = members[a];
        const float *x = X + (int64_t)v * ld;
        double acc = 0.0;
        for (int i = 0; i < d; ++i) {
            double t = (double)x[i] - mean[i];
            acc += t * t;
        }
        if (acc < bestd || (acc == bestd && v < best)) {
            bestd = acc;
            best = v;
        }
    }
    return best;
}

int64_t mark_from(const std::vector<int32_t> &adj, int R, int64_t n, int32_t src, std::vector<uint8_t> &mark,
                  std::vector<int32_t> &newly)
{
    newly.clear();
    if (mark[src]) return 0;
    mark[src] = 1;
    newly.push_back(src);
    for (size_t h = 0; h < newly.size(); ++h) {
        const int32_t v = newly[h];
        for (int r = 0; r < R; ++r) {
            const int32_t u = adj[(int64_t)v * R + r];
            if (u < 0 || u >= n || mark[u]) continue;
            mark[u] = 1;
            newly.push_back(u);
        }
    }
    return (int64_t)newly.size();
}

int64_t uf_find(std::vector<int64_t> &par, int64_t x)
{
    while (par[x] != x) {
        par[x] = par[par[x]];
        x = par[x];
    }
    return x;
}

// device buffer that frees itself
template <typename T>
struct DevBuf {
    T *p = nullptr;
    hipError_t alloc(size_t count) { return hipMalloc(reinterpret_cast<void **>(&p), sizeof(T) * (count ? count : 1)); }
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

int medoid_device(const float *base, int64_t n, int d, int64_t ld, int32_t *out, hipStream_t s)
{
    const int64_t nchunks = (n + MED_CHUNK - 1) / MED_CHUNK;
    const int64_t nblk = (n + 255) / 256;
    DevBuf<double> part, mean, bestd;
    DevBuf<int64_t> besti;
    if (part.alloc(nchunks * d) != hipSuccess || mean.alloc(d) != hipSuccess || bestd.alloc(nblk) != hipSuccess ||
        besti.alloc(nblk) != hipSuccess)
        return set_error(SA_ENOMEM, "medoid: device allocation failed");
    hipLaunchKernelGGL(colsum_partial, dim3((unsigned)nchunks), dim3(128), 0, s, base, n, d, ld, part.p);
    hipLaunchKernelGGL(colsum_final, dim3((d + 127) / 128), dim3(128), 0, s, part.p, nchunks, d, n, mean.p);
    hipLaunchKernelGGL(dist_to_mean, dim3((unsigned)nblk), dim3(256), 0, s, base, n, d, ld, mean.p, bestd.p, besti.p);
    SA_HIP(hipGetLastError());
    std::vector<double> hd(nblk);
    std::vector<int64_t> hi(nblk);
    SA_HIP(hipMemcpyAsync(hd.data(), bestd.p, sizeof(double) * nblk, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(hi.data(), besti.p, sizeof(int64_t) * nblk, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    double bd = INFINITY;
    int64_t bi = -1;
    for (int64_t b = 0; b < nblk; ++b)
        if (hd[b] < bd || (hd[b] == bd && hi[b] < bi)) {
            bd = hd[b];
            bi = hi[b];
        }
    *out = (int32_t)bi;
    return SA_OK;
}

int prune_device(const float *base, int64_t n, int d, int64_t ld, int metric, const int32_t *cand, int kc, int R,
                 int mode, int32_t *adj, hipStream_t s)
{
    if (n == 0) return SA_OK;
    hipLaunchKernelGGL(prune_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, base, n, d, ld, metric, cand, kc,
                       R, mode, adj);
    SA_HIP(hipGetLastError());
    return SA_OK;
}

int reverse_edges_device(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj_dev, int R,
                         int64_t *added_out, hipStream_t s)
{
    const int64_t ne = n * R;
    DevBuf<float> dd;
    if (dd.alloc(ne) != hipSuccess) return set_error(SA_ENOMEM, "reverse edges: device allocation failed");
    hipLaunchKernelGGL(edge_dists, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, base, n, d, ld, metric,
                       adj_dev, R, dd.p);
    SA_HIP(hipGetLastError());
    std::vector<int32_t> snap((size_t)ne);
    std::vector<float> ed((size_t)ne);
    SA_HIP(hipMemcpyAsync(snap.data(), adj_dev, sizeof(int32_t) * ne, hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(ed.data(), dd.p, sizeof(float) * ne, hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));
    // in-edges grouped by target, each group in key order (d(c, p), p)
    std::vector<int64_t> start(n + 1, 0);
    for (int64_t e = 0; e < ne; ++e)
        if (snap[e] >= 0 && snap[e] < n) start[snap[e] + 1]++;
    for (int64_t c = 0; c < n; ++c) start[c + 1] += start[c];
    struct In {
        float d;
        int32_t p;
    };
    std::vector<In> in((size_t)start[n]);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t e = 0; e < ne; ++e) {
            const int32_t c = snap[e];
            if (c >= 0 && c < n) in[fill[c]++] = {ed[e], (int32_t)(e / R)};
        }
    }
    std::vector<int32_t> adj(snap);
    int64_t added = 0;
    for (int64_t c = 0; c < n; ++c) {
        int deg = 0;
        while (deg < R && adj[c * R + deg] >= 0) ++deg;
        if (deg >= R || start[c + 1] == start[c]) continue;
        In *b = in.data() + start[c], *e = in.data() + start[c + 1];
        std::sort(b, e, [](const In &x, const In &y) { return key_less_host(x.d, x.p, y.d, y.p); });
        for (In *it = b; it != e && deg < R; ++it) {
            bool dup = false;
            for (int r = 0; r < deg; ++r)
                if (adj[c * R + r] == it->p) {
                    dup = true;
                    break;
                }
            if (dup) continue;
            adj[c * R + deg++] = it->p;
            ++added;
        }
    }
    SA_HIP(hipMemcpyAsync(adj_dev, adj.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice, s));
    SA_HIP(hipStreamSynchronize(s));
    if (added_out) *added_out = added;
    return SA_OK;
}

int repair_device(const float *base, int64_t n, int d, int64_t ld, int metric, int32_t *adj_dev, int R,
                  int32_t entry, int keep_local, int hubs, int hub_keep_local, int64_t *bridges_out,
                  int64_t *ncomp_out, hipStream_t s)
{
    std::vector<int32_t> adj((size_t)n * R);
    std::vector<float> X((size_t)n * ld);
    SA_HIP(hipMemcpyAsync(adj.data(), adj_dev, sizeof(int32_t) * adj.size(), hipMemcpyDeviceToHost, s));
    SA_HIP(hipMemcpyAsync(X.data(), base, sizeof(float) * X.size(), hipMemcpyDeviceToHost, s));
    SA_HIP(hipStreamSynchronize(s));

    // (1) weakly connected components, numbered by smallest member; medoid of each
    std::vector<int64_t> par(n);
    std::iota(par.begin(), par.end(), 0);
    for (int64_t v = 0; v < n; ++v)
        for (int r = 0; r < R; ++r) {
            const int32_t u = adj[v * R + r];
            if (u < 0) continue;
            int64_t a = uf_find(par, v), b = uf_find(par, u);
            if (a != b) {
                if (a < b) par[b] = a;
                else par[a] = b;
            }
        }
    std::vector<int64_t> comp(n), root_comp(n, -1);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t rt = uf_find(par, i);
        if (root_comp[rt] < 0) root_comp[rt] = nc++;
        comp[i] = root_comp[rt];
    }
    std::vector<int64_t> start(nc + 1, 0);
    for (int64_t i = 0; i < n; ++i) start[comp[i] + 1]++;
    for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
    std::vector<int32_t> members(n);
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t i = 0; i < n; ++i) members[fill[comp[i]]++] = (int32_t)i;
    }
    std::vector<int32_t> rep(nc);
    for (int64_t c = 0; c < nc; ++c) rep[c] = host_medoid(X.data(), ld, d, members.data() + start[c], start[c + 1] - start[c]);
    if (ncomp_out) *ncomp_out = nc;

    // (2) gateway rows for the representatives, the entry and the hubs (the vertices
    // nearest to the mean of all rows)
    std::vector<uint8_t> is_rep(n, 0);
    for (int64_t c = 0; c < nc; ++c) is_rep[rep[c]] = 1;
    std::vector<int32_t> hub;
    if (nc > 1) {
        if (!is_rep[entry]) hub.push_back(entry);
        if (hubs > 1) {
            std::vector<double> mean(d, 0.0);
            for (int64_t v = 0; v < n; ++v)
                for (int i = 0; i < d; ++i) mean[i] += (double)X[(size_t)v * ld + i];
            for (int i = 0; i < d; ++i) mean[i] /= (double)n;
            struct H {
                double d;
                int32_t v;
            };
            std::vector<H> hv;
            hv.reserve(n);
            for (int64_t v = 0; v < n; ++v) {
                if (is_rep[v] || v == entry) continue;
                double acc = 0.0;
                for (int i = 0; i < d; ++i) {
                    double t = (double)X[(size_t)v * ld + i] - mean[i];
                    acc += t * t;
                }
                hv.push_back({acc, (int32_t)v});
            }
            const size_t take = std::min(hv.size(), (size_t)(hubs - 1));
            std::partial_sort(hv.begin(), hv.begin() + take, hv.end(),
                              [](const H &x, const H &y) { return x.d < y.d || (x.d == y.d && x.v < y.v); });
            for (size_t j = 0; j < take; ++j) hub.push_back(hv[j].v);
        }
    }
    const int64_t nsrc = nc > 1 ? nc + (int64_t)hub.size() : 0;
    if (nsrc > 0) {
        // representative-to-representative distances, used by the occlusion test
        std::vector<float> rd((size_t)nc * nc);
        for (int64_t i = 0; i < nc; ++i)
            for (int64_t j = 0; j < nc; ++j)
                rd[(size_t)i * nc + j] = host_dist(&X[(size_t)rep[i] * ld], &X[(size_t)rep[j] * ld], d, metric);
        std::vector<int32_t> links((size_t)nsrc * R, -1);
        std::vector<int> kept_local(nsrc);
        for (int64_t a = 0; a < nsrc; ++a) {
            const int32_t v = a < nc ? rep[a] : hub[a - nc];
            const int kl = a < nc ? keep_local : hub_keep_local;
            kept_local[a] = kl;
            const int cap = R - kl;
            if (cap <= 0) continue;
            struct Cd {
                float d;
                int32_t id;
                int32_t c;
                bool used;
            };
            std::vector<Cd> cand;
            cand.reserve(nc);
            for (int64_t c = 0; c < nc; ++c) {
                if (rep[c] == v) continue;
                cand.push_back({host_dist(&X[(size_t)v * ld], &X[(size_t)rep[c] * ld], d, metric), rep[c], (int32_t)c,
                                false});
            }
            std::sort(cand.begin(), cand.end(), [](const Cd &x, const Cd &y) { return key_less_host(x.d, x.id, y.d, y.id); });
            int32_t *out = &links[(size_t)a * R];
            std::vector<int32_t> kc;
            for (auto &c : cand) {
                if ((int)kc.size() >= cap) break;
                bool keep = true;
                for (int32_t x : kc)
                    if (rd[(size_t)x * nc + c.c] < c.d) {
                        keep = false;
                        break;
                    }
                if (keep) {
                    kc.push_back(c.c);
                    c.used = true;
                }
            }
            int kept = 0;
            for (int32_t x : kc) out[kept++] = rep[x];
            for (auto &c : cand) {
                if (kept >= cap) break;
                if (!c.used) out[kept++] = c.id;
            }
        }
        for (int64_t a = 0; a < nsrc; ++a) {
            const int32_t v = a < nc ? rep[a] : hub[a - nc];
            int32_t *rw = &adj[(int64_t)v * R];
            const int32_t *lk = &links[(size_t)a * R];
            std::vector<int32_t> nr;
            for (int r = 0; r < R && (int)nr.size() < kept_local[a]; ++r) {
                const int32_t u = rw[r];
                if (u < 0) continue;
                if (std::find(lk, lk + R, u) != lk + R) continue;
                nr.push_back(u);
            }
            for (int x = 0; x < R; ++x)
                if (lk[x] >= 0) nr.push_back(lk[x]);
            for (int r = 0; r < R; ++r) rw[r] = r < (int)nr.size() ? nr[r] : -1;
        }
    }

    // (3) reachability: bridge every unreachable vertex, in id order, from the nearest
    // reachable vertex with a free slot
    std::vector<uint8_t> mark(n, 0);
    std::vector<int32_t> newly;
    mark_from(adj, R, n, entry, mark, newly);
    std::vector<int32_t> deg(n);
    for (int64_t v = 0; v < n; ++v) {
        int c = 0;
        for (int r = 0; r < R; ++r) c += adj[v * R + r] >= 0;
        deg[v] = c;
    }
    int64_t added = 0;
    int64_t first_unmarked = 0;
    while (first_unmarked < n && mark[first_unmarked]) ++first_unmarked;
    if (first_unmarked < n) {
        // In id order, as one at a time, but the searches go out in windows of WIN vertices:
        // one launch finds, for each, the nearest vertex with a free slot among those marked
        // when the window starts; processing the window in order, each answer is corrected
        // with the vertices marked since (the same distance arithmetic on the host), and
        // found again alone if its vertex has no free slot left.  The edges are those the
        // one-at-a-time loop adds.  A window ends early once many vertices were marked in it.
        constexpr int WIN = 256;
        constexpr size_t MAX_NEW = 4096;
        DevBuf<uint8_t> dmask;
        DevBuf<int32_t> ddeg, dus;
        DevBuf<unsigned long long> dres;
        if (dmask.alloc(n) != hipSuccess || ddeg.alloc(n) != hipSuccess || dus.alloc(WIN) != hipSuccess ||
            dres.alloc(WIN) != hipSuccess)
            return set_error(SA_ENOMEM, "repair: device allocation failed");
        std::vector<int32_t> us;
        std::vector<unsigned long long> res(WIN);
        std::vector<int32_t> since;   // vertices marked since the window's searches
        // nearest marked vertex with a free slot for each of us, under the current marks and degrees
        auto search = [&](const std::vector<int32_t> &q) -> int {
            SA_HIP(hipMemcpyAsync(dmask.p, mark.data(), n, hipMemcpyHostToDevice, s));
            SA_HIP(hipMemcpyAsync(ddeg.p, deg.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
            SA_HIP(hipMemcpyAsync(dus.p, q.data(), sizeof(int32_t) * q.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(fill_u64_n, dim3(1), dim3(WIN), 0, s, dres.p, (int64_t)q.size(),
                               (unsigned long long)KEY_EMPTY);
            hipLaunchKernelGGL(nearest_marked_batch, dim3((unsigned)((n + 255) / 256), (unsigned)q.size()), dim3(256),
                               0, s, base, n, d, ld, metric, dmask.p, ddeg.p, R, dus.p, dres.p);
            SA_HIP(hipGetLastError());
            SA_HIP(hipMemcpyAsync(res.data(), dres.p, sizeof(unsigned long long) * q.size(), hipMemcpyDeviceToHost, s));
            SA_HIP(hipStreamSynchronize(s));
            return SA_OK;
        };
        int64_t next = first_unmarked;
        while (next < n) {
            us.clear();
            for (int64_t u = next; u < n && (int)us.size() < WIN; ++u)
                if (!mark[u]) us.push_back((int32_t)u);
            if (us.empty()) break;
            int rc = search(us);
            if (rc != SA_OK) return rc;
            since.clear();
            next = (int64_t)us.back() + 1;
            for (size_t j = 0; j < us.size(); ++j) {
                const int32_t u = us[j];
                if (mark[u]) continue;
                if (since.size() > MAX_NEW) {   // many new candidates: search the rest of the window again
                    next = u;
                    break;
                }
                // the window's answer is the best over the vertices marked at its start; those
                // that filled up since cannot be taken, and those marked since are candidates
                unsigned long long best = res[j];
                if (best != KEY_EMPTY && deg[key_id(best)] >= R) {
                    const std::vector<unsigned long long> saved(res);
                    if ((rc = search(std::vector<int32_t>{u})) != SA_OK) return rc;
                    best = res[0];
                    res = saved;
                } else {
                    for (int32_t w : since)
                        if (deg[w] < R) {
                            const unsigned long long k =
                                make_key(host_dist(&X[(size_t)w * ld], &X[(size_t)u * ld], d, metric), w);
                            if (k < best) best = k;
                        }
                }
                if (best == KEY_EMPTY) return set_error(SA_ECAPACITY, "repair: no reachable vertex has a free slot");
                const int32_t r = key_id(best);
                adj[(int64_t)r * R + deg[r]] = u;
                deg[r]++;
                ++added;
                mark_from(adj, R, n, u, mark, newly);
                since.insert(since.end(), newly.begin(), newly.end());
            }
        }
    }
    SA_HIP(hipMemcpyAsync(adj_dev, adj.data(), sizeof(int32_t) * adj.size(), hipMemcpyHostToDevice, s));
    SA_HIP(hipStreamSynchronize(s));
    if (bridges_out) *bridges_out = added;
    return SA_OK;
}

}  // namespace sa

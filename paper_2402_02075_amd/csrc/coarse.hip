// Coarse levels: random-hash agglomeration, first-order KFVS, restriction,
// forcing term, coarse sweeps, prolongation and the V-cycle driver.
//
// Paper Sec. 4.1 (Algorithm 1, cell coarsening): face hash
// h = [23 (N_l + N_r) + N_l N_r] % N_f, first occurrence of each hash value
// selects a face, skewness check against the virtual centre, merge, coarse
// volume and centre as sums.  Sec. 4.2: restriction of the state (volume
// weighted) and of the residual (sum), forcing term, coarse explicit update,
// correction, three-level V-cycle.  Secs. 1 and 6: first-order KFVS with local
// time stepping on the coarse levels.
//
// Parallel form of Algorithm 1 (equal to the sequential loop):
//  - first occurrence: atomicMin of the face index into a table indexed by hash;
//  - greedy matching in ascending face order = repeated rounds in which a live
//    face is taken when it is the smallest live face at both of its cells
//    (such a face has every smaller neighbouring face already dead, i.e. it
//    would be taken by the sequential loop); cells of taken faces kill their
//    other faces; rounds end when no face is live;
//  - relabelling by an exclusive scan over surviving representatives keeps the
//    numbering by smallest member id;
//  - coarse pairs by a stable radix sort of (pair key, face index), each pair's
//    area, moment and area vector summed sequentially in face order.
// The skewness predicate uses +, -, * only in a fixed association order with
// contraction off, so it takes bit-identical decisions on identical inputs.
#include <hipcub/hipcub.hpp>
#include <parallel/algorithm>

#include "common.hpp"
#include "gks_device.hpp"
#include "bc_device.hpp"

namespace cgks {

// ---------------------------------------------------------------- agglomeration kernels
__global__ void k_fill_i32(int32_t *p, int32_t v, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_hash_min(int64_t m, uint64_t seed, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                           int32_t *__restrict__ table)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint64_t a = (uint64_t)pa[j], b = (uint64_t)pb[j];
    const uint64_t h = (23ull * seed * (a + b) + a * b) % (uint64_t)m;
    atomicMin(&table[h], (int32_t)j);
}

__device__ __noinline__ bool skew_accept(double Va, double Vb, const double *Pa, const double *Pb, double S,
                                         const double *M, const double *A, double delta, double smin)
{
#pragma clang fp contract(off)
    const double V = Va + Vb;
    const double P0 = Pa[0] + Pb[0], P1 = Pa[1] + Pb[1], P2 = Pa[2] + Pb[2];
    const double e0 = V * M[0] - S * P0, e1 = V * M[1] - S * P1, e2 = V * M[2] - S * P2;
    const double ee = e0 * e0 + e1 * e1 + e2 * e2;
    const double d2 = delta * delta;
    const double d6 = d2 * d2 * d2;
    const double V2 = V * V, V4 = V2 * V2, V8 = V4 * V4;
    const double S2 = S * S, S6 = S2 * S2 * S2;
    if (ee * ee * ee <= d6 * V8 * S6) return true;
    const double ea = e0 * A[0] + e1 * A[1] + e2 * A[2];
    const double aa = A[0] * A[0] + A[1] * A[1] + A[2] * A[2];
    const double s2 = smin * smin;
    return ea * ea >= s2 * ee * aa;
}

__global__ void k_select(int64_t m, uint64_t seed, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                         const int32_t *__restrict__ table, const double *__restrict__ V, const double *__restrict__ P,
                         const double *__restrict__ S, const double *__restrict__ M, const double *__restrict__ A,
                         double delta, double smin, uint8_t *__restrict__ live, int32_t *__restrict__ cnt)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint64_t a = (uint64_t)pa[j], b = (uint64_t)pb[j];
    const uint64_t h = (23ull * seed * (a + b) + a * b) % (uint64_t)m;
    uint8_t ok = 0;
    if (table[h] == (int32_t)j) {
        atomicAdd(&cnt[0], 1);
        if (skew_accept(V[a], V[b], &P[3 * a], &P[3 * b], S[j], &M[3 * j], &A[3 * j], delta, smin)) {
            ok = 1;
            atomicAdd(&cnt[1], 1);
        }
    }
    live[j] = ok;
}

__global__ void k_match_min(int64_t m, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                            const uint8_t *__restrict__ live, int32_t *__restrict__ best)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || !live[j]) return;
    atomicMin(&best[pa[j]], (int32_t)j);
    atomicMin(&best[pb[j]], (int32_t)j);
}

__global__ void k_match_take(int64_t m, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                             uint8_t *__restrict__ live, const int32_t *__restrict__ best, int32_t *__restrict__ mate,
                             int32_t *__restrict__ partner, uint8_t *__restrict__ matched, int32_t *__restrict__ cnt)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || !live[j]) return;
    const int a = pa[j], b = pb[j];
    if (best[a] == (int32_t)j && best[b] == (int32_t)j) {
        mate[b] = a;
        partner[a] = b;
        matched[a] = 1;
        matched[b] = 1;
        atomicAdd(&cnt[2], 1);
    }
}

__global__ void k_match_kill(int64_t m, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                             uint8_t *__restrict__ live, const uint8_t *__restrict__ matched, int32_t *__restrict__ cnt)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m || !live[j]) return;
    if (matched[pa[j]] || matched[pb[j]]) live[j] = 0;
    else atomicAdd(&cnt[3], 1);
}

__global__ void k_surv(int64_t n, const int32_t *__restrict__ mate, int32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = mate[i] < 0 ? 1 : 0;
}

__global__ void k_newid(int64_t n, const int32_t *__restrict__ mate, int32_t *__restrict__ newid)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && mate[i] >= 0) newid[i] = newid[mate[i]];
}

__global__ void k_new_geom(int64_t n, const int32_t *__restrict__ mate, const int32_t *__restrict__ partner,
                           const int32_t *__restrict__ newid, const double *__restrict__ V, const double *__restrict__ P,
                           double *__restrict__ Vo, double *__restrict__ Po)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || mate[i] >= 0) return;
    const int k = newid[i];
    const int b = partner[i];
    if (b >= 0) {
        Vo[k] = V[i] + V[b];
#pragma unroll
        for (int d = 0; d < 3; ++d) Po[3 * k + d] = P[3 * i + d] + P[3 * b + d];
    } else {
        Vo[k] = V[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) Po[3 * k + d] = P[3 * i + d];
    }
}

__global__ void k_compose(int64_t n, int32_t *__restrict__ f2c, const int32_t *__restrict__ newid)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f2c[i] = newid[f2c[i]];
}

__global__ void k_iota(int64_t n, int32_t *p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = (int32_t)i;
}

// key of the relabelled pair (min, max) << ; dropped pairs get the largest key
__global__ void k_pair_keys(int64_t m, const int32_t *__restrict__ pa, const int32_t *__restrict__ pb,
                            const int32_t *__restrict__ newid, uint64_t *__restrict__ key, int32_t *__restrict__ idx)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint32_t a = (uint32_t)newid[pa[j]], b = (uint32_t)newid[pb[j]];
    key[j] = a == b ? ~0ull : ((uint64_t)(a < b ? a : b) << 32) | (uint64_t)(a < b ? b : a);
    idx[j] = (int32_t)j;
}

__global__ void k_seg_heads(int64_t m, const uint64_t *__restrict__ key, int32_t *__restrict__ head)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    head[j] = (key[j] != ~0ull && (j == 0 || key[j] != key[j - 1])) ? 1 : 0;
}

__global__ void k_seg_start(int64_t m, const int32_t *__restrict__ head, const int32_t *__restrict__ segid,
                            int32_t *__restrict__ start)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m && head[j]) start[segid[j]] = (int32_t)j;
}

// one thread per coarse pair: sequential sums in ascending face index
__global__ void k_seg_sum(int64_t nseg, int64_t m, const int32_t *__restrict__ start, const uint64_t *__restrict__ key,
                          const int32_t *__restrict__ idx, const int32_t *__restrict__ pa,
                          const int32_t *__restrict__ newid, const double *__restrict__ S, const double *__restrict__ M,
                          const double *__restrict__ A, int32_t *__restrict__ pao, int32_t *__restrict__ pbo,
                          double *__restrict__ So, double *__restrict__ Mo, double *__restrict__ Ao)
{
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const int64_t b = start[g];
    const uint64_t k0 = key[b];
    double s = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0, a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int64_t q = b; q < m && key[q] == k0; ++q) {
        const int j = idx[q];
        const uint32_t lo = (uint32_t)(k0 >> 32);
        const bool rev = (uint32_t)newid[pa[j]] != lo;
        s += S[j];
        m0 += M[3 * j];
        m1 += M[3 * j + 1];
        m2 += M[3 * j + 2];
        a0 += rev ? -A[3 * j] : A[3 * j];
        a1 += rev ? -A[3 * j + 1] : A[3 * j + 1];
        a2 += rev ? -A[3 * j + 2] : A[3 * j + 2];
    }
    pao[g] = (int32_t)(k0 >> 32);
    pbo[g] = (int32_t)(k0 & 0xffffffffu);
    So[g] = s;
    Mo[3 * g] = m0;
    Mo[3 * g + 1] = m1;
    Mo[3 * g + 2] = m2;
    Ao[3 * g] = a0;
    Ao[3 * g + 1] = a1;
    Ao[3 * g + 2] = a2;
}

// ---------------------------------------------------------------- agglomeration driver
namespace {
struct Scratch {
    DBuf<int32_t> table, best, mate, partner, newid, flag, cnt, idx, idx2, head, segid, start;
    DBuf<uint8_t> live, matched;
    DBuf<uint64_t> key, key2;
    DBuf<uint8_t> tmp;
};

void scan_excl(Scratch &s, const int32_t *in, int32_t *out, int64_t n, hipStream_t st)
{
    size_t bytes = 0;
    CGKS_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, bytes, in, out, (int)n, st));
    s.tmp.ensure(bytes + 1);
    CGKS_HIP(hipcub::DeviceScan::ExclusiveSum(s.tmp.p, bytes, in, out, (int)n, st));
}
}  // namespace

static inline dim3 G1(int64_t n) { return dim3(blocks_for(n > 0 ? n : 1, 256)); }

void agglomerate_graph(cgks_ctx *c, int64_t n, const double *V, const double *P, int64_t m, const int32_t *pa,
                       const int32_t *pb, const double *S, const double *M, const double *A, int passes, int32_t *f2c,
                       double *Vc, double *Pc, int64_t *n_coarse, int64_t *m_coarse, int64_t *stats, int32_t *pa_out,
                       int32_t *pb_out, double *S_out, double *M_out, double *A_out)
{
    hipStream_t st = c->stream;
    const dim3 B(256);
    Scratch s;
    // current graph buffers (ping-pong)
    DBuf<double> cV, cP, cS, cM, cA, nV, nP, nS, nM, nA;
    DBuf<int32_t> ca, cb, na, nb;
    cV.alloc(n);
    cP.alloc(3 * n);
    cS.alloc(m + 1);
    cM.alloc(3 * m + 3);
    cA.alloc(3 * m + 3);
    ca.alloc(m + 1);
    cb.alloc(m + 1);
    nV.alloc(n);
    nP.alloc(3 * n);
    nS.alloc(m + 1);
    nM.alloc(3 * m + 3);
    nA.alloc(3 * m + 3);
    na.alloc(m + 1);
    nb.alloc(m + 1);
    CGKS_HIP(hipMemcpyAsync(cV.p, V, 8 * n, hipMemcpyDeviceToDevice, st));
    CGKS_HIP(hipMemcpyAsync(cP.p, P, 24 * n, hipMemcpyDeviceToDevice, st));
    if (m) {
        CGKS_HIP(hipMemcpyAsync(cS.p, S, 8 * m, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(cM.p, M, 24 * m, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(cA.p, A, 24 * m, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(ca.p, pa, 4 * m, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(cb.p, pb, 4 * m, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_iota, G1(n), B, 0, st, n, f2c);
    s.table.alloc(m + 1);
    s.best.alloc(n);
    s.mate.alloc(n);
    s.partner.alloc(n);
    s.newid.alloc(n);
    s.flag.alloc(n);
    s.cnt.alloc(8);
    s.live.alloc(m + 1);
    s.matched.alloc(n);
    s.key.alloc(m + 1);
    s.key2.alloc(m + 1);
    s.idx.alloc(m + 1);
    s.idx2.alloc(m + 1);
    s.head.alloc(m + 1);
    s.segid.alloc(m + 1);
    s.start.alloc(m + 1);
    int64_t cn = n, cm = m;
    for (int pass = 0; pass < passes; ++pass) {
        int32_t hc[4] = {0, 0, 0, 0};
        CGKS_HIP(hipMemcpyAsync(s.cnt.p, hc, sizeof(hc), hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_fill_i32, G1(cn), B, 0, st, s.mate.p, -1, cn);
        hipLaunchKernelGGL(k_fill_i32, G1(cn), B, 0, st, s.partner.p, -1, cn);
        CGKS_HIP(hipMemsetAsync(s.matched.p, 0, cn, st));
        if (cm > 0) {
            hipLaunchKernelGGL(k_fill_i32, G1(cm), B, 0, st, s.table.p, INT32_MAX, cm);
            hipLaunchKernelGGL(k_hash_min, G1(cm), B, 0, st, cm, (uint64_t)c->prm.seed, ca.p, cb.p, s.table.p);
            hipLaunchKernelGGL(k_select, G1(cm), B, 0, st, cm, (uint64_t)c->prm.seed, ca.p, cb.p, s.table.p, cV.p, cP.p,
                               cS.p, cM.p, cA.p, c->prm.skew_delta, c->prm.skew_sin, s.live.p, s.cnt.p);
            for (int round = 0;; ++round) {
                hipLaunchKernelGGL(k_fill_i32, G1(cn), B, 0, st, s.best.p, INT32_MAX, cn);
                hipLaunchKernelGGL(k_match_min, G1(cm), B, 0, st, cm, ca.p, cb.p, s.live.p, s.best.p);
                hipLaunchKernelGGL(k_match_take, G1(cm), B, 0, st, cm, ca.p, cb.p, s.live.p, s.best.p, s.mate.p,
                                   s.partner.p, s.matched.p, s.cnt.p);
                int32_t zero = 0;
                CGKS_HIP(hipMemcpyAsync(s.cnt.p + 3, &zero, 4, hipMemcpyHostToDevice, st));
                hipLaunchKernelGGL(k_match_kill, G1(cm), B, 0, st, cm, ca.p, cb.p, s.live.p, s.matched.p, s.cnt.p);
                int32_t alive = 0;
                CGKS_HIP(hipMemcpyAsync(&alive, s.cnt.p + 3, 4, hipMemcpyDeviceToHost, st));
                CGKS_HIP(hipStreamSynchronize(st));
                if (alive == 0) break;
                if (round > 100000) throw Error{CGKS_E_DEVICE, "matching rounds did not terminate"};
            }
        }
        CGKS_HIP(hipMemcpyAsync(hc, s.cnt.p, sizeof(hc), hipMemcpyDeviceToHost, st));
        // relabel: exclusive scan over representatives
        hipLaunchKernelGGL(k_surv, G1(cn), B, 0, st, cn, s.mate.p, s.flag.p);
        scan_excl(s, s.flag.p, s.newid.p, cn, st);
        int32_t lastf = 0, lastid = 0;
        CGKS_HIP(hipMemcpyAsync(&lastf, s.flag.p + cn - 1, 4, hipMemcpyDeviceToHost, st));
        CGKS_HIP(hipMemcpyAsync(&lastid, s.newid.p + cn - 1, 4, hipMemcpyDeviceToHost, st));
        hipLaunchKernelGGL(k_newid, G1(cn), B, 0, st, cn, s.mate.p, s.newid.p);
        hipLaunchKernelGGL(k_new_geom, G1(cn), B, 0, st, cn, s.mate.p, s.partner.p, s.newid.p, cV.p, cP.p, nV.p, nP.p);
        hipLaunchKernelGGL(k_compose, G1(n), B, 0, st, n, f2c, s.newid.p);
        CGKS_HIP(hipStreamSynchronize(st));
        const int64_t nn = (int64_t)lastid + lastf;
        // coarse pairs
        int64_t nm = 0;
        if (cm > 0) {
            hipLaunchKernelGGL(k_pair_keys, G1(cm), B, 0, st, cm, ca.p, cb.p, s.newid.p, s.key.p, s.idx.p);
            size_t bytes = 0;
            CGKS_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, s.key.p, s.key2.p, s.idx.p, s.idx2.p, (int)cm, 0,
                                                        64, st));
            s.tmp.ensure(bytes + 1);
            CGKS_HIP(hipcub::DeviceRadixSort::SortPairs(s.tmp.p, bytes, s.key.p, s.key2.p, s.idx.p, s.idx2.p, (int)cm,
                                                        0, 64, st));
            hipLaunchKernelGGL(k_seg_heads, G1(cm), B, 0, st, cm, s.key2.p, s.head.p);
            scan_excl(s, s.head.p, s.segid.p, cm, st);
            int32_t lh = 0, ls = 0;
            CGKS_HIP(hipMemcpyAsync(&lh, s.head.p + cm - 1, 4, hipMemcpyDeviceToHost, st));
            CGKS_HIP(hipMemcpyAsync(&ls, s.segid.p + cm - 1, 4, hipMemcpyDeviceToHost, st));
            CGKS_HIP(hipStreamSynchronize(st));
            nm = (int64_t)ls + lh;
            hipLaunchKernelGGL(k_seg_start, G1(cm), B, 0, st, cm, s.head.p, s.segid.p, s.start.p);
            hipLaunchKernelGGL(k_seg_sum, G1(nm), B, 0, st, nm, cm, s.start.p, s.key2.p, s.idx2.p, ca.p, s.newid.p,
                               cS.p, cM.p, cA.p, na.p, nb.p, nS.p, nM.p, nA.p);
        }
        if (stats) {
            stats[4 * pass + 0] = hc[0];
            stats[4 * pass + 1] = hc[1];
            stats[4 * pass + 2] = hc[2];
            stats[4 * pass + 3] = nm;
        }
        std::swap(cV.p, nV.p);
        std::swap(cP.p, nP.p);
        std::swap(cS.p, nS.p);
        std::swap(cM.p, nM.p);
        std::swap(cA.p, nA.p);
        std::swap(ca.p, na.p);
        std::swap(cb.p, nb.p);
        cn = nn;
        cm = nm;
    }
    CGKS_HIP(hipMemcpyAsync(Vc, cV.p, 8 * cn, hipMemcpyDeviceToDevice, st));
    CGKS_HIP(hipMemcpyAsync(Pc, cP.p, 24 * cn, hipMemcpyDeviceToDevice, st));
    if (pa_out && cm) {
        CGKS_HIP(hipMemcpyAsync(pa_out, ca.p, 4 * cm, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(pb_out, cb.p, 4 * cm, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(S_out, cS.p, 8 * cm, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(M_out, cM.p, 24 * cm, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(A_out, cA.p, 24 * cm, hipMemcpyDeviceToDevice, st));
    }
    CGKS_HIP(hipStreamSynchronize(st));
    *n_coarse = cn;
    *m_coarse = cm;
}

// ---------------------------------------------------------------- hierarchy
__global__ void k_interleaved_to_soa(int64_t m, const double *__restrict__ in, double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
#pragma unroll
    for (int d = 0; d < 3; ++d) out[d * m + j] = in[3 * j + d];
}

namespace {
// host description of a graph level before upload
struct HostGraph {
    std::vector<int32_t> a, b;     // candidate pairs
    std::vector<int32_t> pera, perb; // periodic pairs (kept out of agglomeration)
    std::vector<double> perA;      // interleaved area vectors of periodic pairs
    std::vector<double> perS;
};

void build_cell_items(Level *L, const std::vector<int32_t> &pa, const std::vector<int32_t> &pb,
                      const std::vector<int32_t> &bown, hipStream_t st)
{
    const int64_t n = L->n, m = (int64_t)pa.size(), nb = (int64_t)bown.size();
    std::vector<int32_t> ptr(n + 1, 0);
    for (int64_t j = 0; j < m; ++j) {
        ptr[pa[j] + 1]++;
        ptr[pb[j] + 1]++;
    }
    for (int64_t k = 0; k < nb; ++k) ptr[bown[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    std::vector<int32_t> item(ptr[n]);
    std::vector<int32_t> fill(n, 0);
    for (int64_t j = 0; j < m; ++j) {
        item[ptr[pa[j]] + fill[pa[j]]++] = (int32_t)(2 * j);
        item[ptr[pb[j]] + fill[pb[j]]++] = (int32_t)(2 * j + 1);
    }
    for (int64_t k = 0; k < nb; ++k) item[ptr[bown[k]] + fill[bown[k]]++] = (int32_t)(-(k + 1));
    L->nnz = ptr[n];
    L->cf_ptr.upload(ptr, st);
    L->cf_item.upload(item, st);
}

void build_c2f(Level *L, const std::vector<int32_t> &f2c, hipStream_t st)
{
    const int64_t n = L->n, nf = (int64_t)f2c.size();
    std::vector<int32_t> ptr(n + 1, 0), idx(nf);
    for (int64_t i = 0; i < nf; ++i) ptr[f2c[i] + 1]++;
    for (int64_t k = 0; k < n; ++k) ptr[k + 1] += ptr[k];
    std::vector<int32_t> fill(n, 0);
    for (int64_t i = 0; i < nf; ++i) idx[ptr[f2c[i]] + fill[f2c[i]]++] = (int32_t)i;
    L->c2f_ptr.upload(ptr, st);
    L->c2f_idx.upload(idx, st);
}
}  // namespace

void build_hierarchy(cgks_ctx *c)
{
    hipStream_t st = c->stream;
    for (Level *l : c->lev) delete l;
    c->lev.assign(1, nullptr);
    const int levels = c->prm.levels;
    if (levels <= 1) return;
    const int64_t N = c->N, F = c->F, Fi = c->Fi;
    // Fine graph in the caller's cell ids (Sec. 4.1: the hash of Eq. (hash value) and the order of
    // Algorithm 1 act on the input numbering): interior, non-periodic faces as pairs a < b of caller
    // ids, sorted lexicographically, area vectors oriented a -> b; volumes and first moments indexed
    // by caller id.  Periodic faces are kept aside (never merged).
    std::vector<int32_t> hfl = c->fl.download(F, st), hfr = c->fr.download(F, st), htag = c->ftag.download(F, st);
    std::vector<double> hsh = c->fshift.download(3 * F, st), hav = c->favec.download(3 * F, st),
                        har = c->farea.download(F, st), hfm = c->fmom.download(3 * F, st);
    std::vector<int32_t> pera, perb;
    std::vector<double> perA, perS;
    struct GPair {
        int32_t a, b, f;
        bool flip;
    };
    std::vector<GPair> gp;
    gp.reserve(Fi);
    for (int64_t f = 0; f < Fi; ++f) {
        const bool per = hsh[f] != 0.0 || hsh[F + f] != 0.0 || hsh[2 * F + f] != 0.0;
        if (per) {
            pera.push_back(hfl[f]);
            perb.push_back(hfr[f]);
            for (int d = 0; d < 3; ++d) perA.push_back(hav[d * F + f]);
            perS.push_back(har[f]);
            continue;
        }
        const int32_t a = (int32_t)c->caller_cell(hfl[f]), b = (int32_t)c->caller_cell(hfr[f]);
        gp.push_back({std::min(a, b), std::max(a, b), (int32_t)f, a > b});
    }
    if (c->permuted)
        __gnu_parallel::sort(gp.begin(), gp.end(),
                             [](const GPair &x, const GPair &y) { return x.a != y.a ? x.a < y.a : x.b < y.b; });
    const int64_t m0 = (int64_t)gp.size();
    std::vector<int32_t> ga(m0), gb(m0);
    std::vector<double> gS(m0 + 1), gM(3 * m0 + 3), gA(3 * m0 + 3);
    for (int64_t j = 0; j < m0; ++j) {
        if (j > 0 && gp[j].a == gp[j - 1].a && gp[j].b == gp[j - 1].b)
            throw Error{CGKS_E_MESH, "two faces between the same pair of cells are not supported by agglomeration"};
        ga[j] = gp[j].a;
        gb[j] = gp[j].b;
        const int32_t f = gp[j].f;
        const double sg = gp[j].flip ? -1.0 : 1.0;
        gS[j] = har[f];
        for (int d = 0; d < 3; ++d) {
            gM[3 * j + d] = hfm[d * F + f];
            gA[3 * j + d] = sg * hav[d * F + f];
        }
    }
    std::vector<int32_t> bown, btag;
    std::vector<double> bA;
    for (int64_t f = Fi; f < F; ++f) {
        bown.push_back(hfl[f]);
        btag.push_back(htag[f]);
    }
    const int64_t nbf = F - Fi;
    // device graph of the current finest level
    int64_t n = N, m = m0;
    DBuf<double> V, P, S, M, A;
    DBuf<int32_t> pa, pb;
    {
        std::vector<double> hv = c->vol.download(N, st), hc = c->cen.download(3 * N, st);
        std::vector<double> gV(N), gP(3 * N);
        for (int64_t i = 0; i < N; ++i) {
            const int64_t o = c->caller_cell(i);
            gV[o] = hv[i];
            for (int d = 0; d < 3; ++d) gP[3 * o + d] = hv[i] * hc[d * N + i];
        }
        V.upload(gV, st);
        P.upload(gP, st);
    }
    S.upload(gS, st);
    M.upload(gM, st);
    A.upload(gA, st);
    pa.upload(ga, st);
    pb.upload(gb, st);
    // fine boundary area vectors (SoA)
    std::vector<double> hbA(3 * nbf);
    for (int64_t k = 0; k < nbf; ++k)
        for (int d = 0; d < 3; ++d) hbA[d * nbf + k] = hav[d * F + Fi + k];
    std::vector<int32_t> comp(N);  // fine -> current level
    for (int64_t i = 0; i < N; ++i) comp[i] = (int32_t)i;
    std::vector<int32_t> cur_pera = pera, cur_perb = perb;
    std::vector<double> cur_perA = perA, cur_perS = perS;
    for (int l = 1; l < levels; ++l) {
        Level *L = new Level();
        c->lev.push_back(L);
        L->nfine = n;
        L->f2c.alloc(n);
        DBuf<double> Vc, Pc, Sc, Mc, Ac;
        DBuf<int32_t> pac, pbc;
        Vc.alloc(n);
        Pc.alloc(3 * n);
        Sc.alloc(m + 1);
        Mc.alloc(3 * m + 3);
        Ac.alloc(3 * m + 3);
        pac.alloc(m + 1);
        pbc.alloc(m + 1);
        int64_t nc = 0, mc = 0;
        agglomerate_graph(c, n, V.p, P.p, m, pa.p, pb.p, S.p, M.p, A.p, c->prm.passes, L->f2c.p, Vc.p, Pc.p, &nc, &mc,
                          nullptr, pac.p, pbc.p, Sc.p, Mc.p, Ac.p);
        L->n = nc;
        std::vector<int32_t> hf2c = L->f2c.download(n, st);
        if (l == 1 && c->permuted) {
            // level 1 is kept indexed by internal fine cells: f2c_internal[i] = f2c_caller[perm[i]]
            std::vector<int32_t> fi(n);
            for (int64_t i = 0; i < n; ++i) fi[i] = hf2c[c->caller_cell(i)];
            hf2c.swap(fi);
            L->f2c.upload(hf2c, st);
        }
        // periodic pairs carried to the coarse level
        std::vector<int32_t> hpa = pac.download(mc, st), hpb = pbc.download(mc, st);
        std::vector<double> hS = Sc.download(mc, st), hA = Ac.download(3 * mc, st);
        std::vector<int32_t> allA = hpa, allB = hpb;
        std::vector<double> allS = hS, allAv = hA;
        for (size_t q = 0; q < cur_pera.size(); ++q) {
            cur_pera[q] = hf2c[cur_pera[q]];
            cur_perb[q] = hf2c[cur_perb[q]];
            allA.push_back(cur_pera[q]);
            allB.push_back(cur_perb[q]);
            allS.push_back(cur_perS[q]);
            for (int d = 0; d < 3; ++d) allAv.push_back(cur_perA[3 * q + d]);
        }
        const int64_t mall = (int64_t)allA.size();
        L->m = mall;
        L->pa.upload(allA, st);
        L->pb.upload(allB, st);
        L->S.upload(allS, st);
        {
            std::vector<double> as(4 * mall + 4);
            for (int64_t j = 0; j < mall; ++j) {
                for (int d = 0; d < 3; ++d) as[4 * j + d] = allAv[3 * j + d];
                as[4 * j + 3] = allS[j];
            }
            L->AS.upload(as, st);
        }
        {
            DBuf<double> tmp;
            tmp.upload(allAv, st);
            L->A.alloc(3 * mall + 3);
            if (mall) hipLaunchKernelGGL(k_interleaved_to_soa, G1(mall), dim3(256), 0, st, mall, tmp.p, L->A.p);
            CGKS_HIP(hipStreamSynchronize(st));
        }
        L->V.alloc(nc);
        L->P.alloc(3 * nc);
        CGKS_HIP(hipMemcpyAsync(L->V.p, Vc.p, 8 * nc, hipMemcpyDeviceToDevice, st));
        CGKS_HIP(hipMemcpyAsync(L->P.p, Pc.p, 24 * nc, hipMemcpyDeviceToDevice, st));
        // boundary faces: fine faces with the coarse owner
        for (int64_t i = 0; i < N; ++i) comp[i] = hf2c[comp[i]];
        std::vector<int32_t> lbown(nbf);
        for (int64_t k = 0; k < nbf; ++k) lbown[k] = comp[bown[k]];
        L->nb = nbf;
        L->bown.upload(lbown, st);
        L->btag.upload(btag, st);
        L->bA.upload(hbA, st);
        build_cell_items(L, allA, allB, lbown, st);
        build_c2f(L, hf2c, st);
        // work buffers
        L->W0.alloc(5 * nc);
        L->W.alloc(5 * nc);
        L->R.alloc(5 * nc);
        L->F.alloc(5 * nc);
        L->Rs.alloc(5 * nc);
        L->dt.alloc(nc);
        L->fflux.alloc(5 * (mall + nbf) + 5);
        // next level's input graph = this level's agglomerated pairs (periodic ones stay aside)
        std::swap(V.p, Vc.p);
        std::swap(P.p, Pc.p);
        std::swap(S.p, Sc.p);
        std::swap(M.p, Mc.p);
        std::swap(A.p, Ac.p);
        std::swap(pa.p, pac.p);
        std::swap(pb.p, pbc.p);
        n = nc;
        m = mc;
        CGKS_HIP(hipStreamSynchronize(st));
    }
}

// ---------------------------------------------------------------- KFVS and transfers
// Rows of a CSR list handled by RG consecutive lanes each: lane g takes items g, g + RG, ...
// and the partial sums meet in a fixed xor tree, so results are deterministic and a level of a
// few ten thousand cells still fills the chip.
constexpr int RG = 8;
template <class T> __device__ __forceinline__ T row_sum(T v)
{
#pragma unroll
    for (int o = RG / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
static inline dim3 GR(int64_t rows) { return dim3(blocks_for((rows > 0 ? rows : 1) * RG, 256)); }

template <class T> struct CoarseArgs {
    int64_t n, m, nb;
    double gam, K;
    const T *W;
    const int32_t *pa, *pb, *bown, *btag;
    const double *A, *bA;
    const BcTable *bc;
    T *fflux;  // [m + nb][5] (face-major: one face's five values together), S n . F
};

// S n . F of coarse face j (pairs j < m, then boundary faces) at the state W, or at W + D when D
// is given (the sum taken in T, as the state-sum kernel takes it).
template <class T> __device__ __forceinline__ void kfvs_face_flux(const CoarseArgs<T> &A, int64_t j, const T *D, T ff[5])
{
    double av[3];
    double wa[5], wb[5];
    if (j < A.m) {
        for (int d = 0; d < 3; ++d) av[d] = A.A[d * A.m + j];
        const int a = A.pa[j], b = A.pb[j];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            wa[q] = double(D ? T(A.W[q * A.n + a] + D[q * A.n + a]) : A.W[q * A.n + a]);
            wb[q] = double(D ? T(A.W[q * A.n + b] + D[q * A.n + b]) : A.W[q * A.n + b]);
        }
    } else {
        const int64_t k = j - A.m;
        for (int d = 0; d < 3; ++d) av[d] = A.bA[d * A.nb + k];
        const int o = A.bown[k];
#pragma unroll
        for (int q = 0; q < 5; ++q) wa[q] = double(D ? T(A.W[q * A.n + o] + D[q * A.n + o]) : A.W[q * A.n + o]);
    }
    const double S = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
    if (S == 0.0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) ff[q] = T(0);
        return;
    }
    const double n[3] = {av[0] / S, av[1] / S, av[2] / S};
    if (j >= A.m) ghost_state(*A.bc, A.btag[j - A.m], n, wa, A.gam, wb);
    double t1[3], t2[3];
    onb(n, t1, t2);
    T la[5], lb[5];
    la[0] = T(wa[0]);
    la[1] = T(wa[1] * n[0] + wa[2] * n[1] + wa[3] * n[2]);
    la[2] = T(wa[1] * t1[0] + wa[2] * t1[1] + wa[3] * t1[2]);
    la[3] = T(wa[1] * t2[0] + wa[2] * t2[1] + wa[3] * t2[2]);
    la[4] = T(wa[4]);
    lb[0] = T(wb[0]);
    lb[1] = T(wb[1] * n[0] + wb[2] * n[1] + wb[3] * n[2]);
    lb[2] = T(wb[1] * t1[0] + wb[2] * t1[1] + wb[3] * t1[2]);
    lb[3] = T(wb[1] * t2[0] + wb[2] * t2[1] + wb[3] * t2[2]);
    lb[4] = T(wb[4]);
    T Fl[5];
    kfvs_local(la, lb, T(A.gam), T(A.K), Fl);
    ff[0] = T(S * double(Fl[0]));
#pragma unroll
    for (int d = 0; d < 3; ++d) ff[1 + d] = T(S * (double(Fl[1]) * n[d] + double(Fl[2]) * t1[d] + double(Fl[3]) * t2[d]));
    ff[4] = T(S * double(Fl[4]));
}

// one thread per coarse face; the state is W, or W + D when D is given
template <class T> __global__ __launch_bounds__(256) void k_kfvs_face(CoarseArgs<T> A, const T *D)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = A.m + A.nb;
    if (j >= tot) return;
    T ff[5];
    kfvs_face_flux(A, j, D, ff);
#pragma unroll
    for (int q = 0; q < 5; ++q) A.fflux[5 * j + q] = ff[q];
}

// Row kernels of a coarse level's first sweep and of its restriction input: the face-flux
// gather of the KFVS residual (same lanes and order as k_kfvs_gather) fused with the per-cell
// work that follows it.
//  FIRST: residual R0 at W0 (A.W), the local step at W0 (as k_coarse_dt), the forcing
//         F = Rs - R0 and the first delta-form sweep D = dt/V Rs.
//  else:  fluxes taken at W0 + D; writes that state (Wout) and Res_2h(W0 + D) + F (Rout).
template <class T, bool FIRST>
__global__ __launch_bounds__(256) void k_kfvs_rows(CoarseArgs<T> A, const T *__restrict__ ff,
                                                   const int32_t *__restrict__ ptr, const int32_t *__restrict__ item,
                                                   const double *__restrict__ AS, const double *__restrict__ V,
                                                   double cfl, double mu, int viscous, const T *__restrict__ Rs,
                                                   const T *__restrict__ D, T *__restrict__ F, T *__restrict__ Dout,
                                                   T *__restrict__ Wout, T *__restrict__ Rout)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / RG;
    const int g = (int)(t % RG);
    const int64_t n = A.n;
    if (i >= n) return;  // whole row groups leave together
    double u = 0, v = 0, w = 0, cs = 0, rho = 1, Vi = 0;
    if (FIRST) {
        rho = double(A.W[i]);
        const double ir = 1.0 / rho;
        u = double(A.W[n + i]) * ir;
        v = double(A.W[2 * n + i]) * ir;
        w = double(A.W[3 * n + i]) * ir;
        const double p = (A.gam - 1.0) * (double(A.W[4 * n + i]) - 0.5 * rho * (u * u + v * v + w * w));
        cs = sqrt(A.gam * p * ir);
        Vi = V[i];
    }
    // the row's own inputs of the epilogue, requested before the face loop so that their latency
    // overlaps it (lane 0 of the row uses them)
    T pre[10];
    if (g == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            if (FIRST) {
                pre[q] = Rs[q * n + i];
            } else {
                pre[q] = A.W[q * n + i] + D[q * n + i];
                pre[5 + q] = F[q * n + i];
            }
        }
    }
    T r[5] = {T(0), T(0), T(0), T(0), T(0)};
    double sum = 0.0;
    for (int k = ptr[i] + g; k < ptr[i + 1]; k += RG) {
        const int it = item[k];
        if (it >= 0) {
            const int j = it >> 1;
            const T s = (it & 1) ? T(1) : T(-1);
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q] += s * ff[5 * j + q];
        } else {
            const int64_t j = A.m + (-it - 1);
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q] -= ff[5 * j + q];
        }
        if (FIRST) {
            double ax, ay, az, sa;
            if (it >= 0) {
                const int j = it >> 1;
                ax = AS[4 * j];
                ay = AS[4 * j + 1];
                az = AS[4 * j + 2];
                sa = AS[4 * j + 3];
            } else {
                const int q = -it - 1;
                ax = A.bA[q];
                ay = A.bA[A.nb + q];
                az = A.bA[2 * A.nb + q];
                sa = sqrt(ax * ax + ay * ay + az * az);
            }
            const double uA = fabs(u * ax + v * ay + w * az);
            const double lam = cs + (viscous ? 2.0 * mu * sa / (rho * Vi) : 0.0);
            sum += uA + lam * sa;
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = row_sum(r[q]);
    if (FIRST) sum = row_sum(sum);
    if (g != 0) return;
    if (FIRST) {
        const T dti = T(cfl * Vi / sum);
        const T h = dti / T(Vi);
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            F[q * n + i] = pre[q] - r[q];
            Dout[q * n + i] = h * pre[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            Wout[q * n + i] = pre[q];
            Rout[q * n + i] = r[q] + pre[5 + q];
        }
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_kfvs_gather(int64_t n, int64_t m, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ item, const T *__restrict__ ff,
                                                     const T *__restrict__ add, T *__restrict__ R)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / RG;
    const int g = (int)(t % RG);
    if (i >= n) return;  // whole row groups leave together
    T ad[5];  // requested before the face loop so its latency overlaps it
    if (g == 0 && add)
#pragma unroll
        for (int q = 0; q < 5; ++q) ad[q] = add[q * n + i];
    T r[5] = {T(0), T(0), T(0), T(0), T(0)};
    for (int k = ptr[i] + g; k < ptr[i + 1]; k += RG) {
        const int it = item[k];
        if (it >= 0) {
            const int j = it >> 1;
            const T s = (it & 1) ? T(1) : T(-1);
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q] += s * ff[5 * j + q];
        } else {
            const int64_t j = m + (-it - 1);
#pragma unroll
            for (int q = 0; q < 5; ++q) r[q] -= ff[5 * j + q];
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = row_sum(r[q]);
    if (g == 0)
#pragma unroll
        for (int q = 0; q < 5; ++q) R[q * n + i] = add ? r[q] + ad[q] : r[q];
}

// local time step on a coarse level
template <class T>
__global__ __launch_bounds__(256) void k_coarse_dt(int64_t n, int64_t m, int64_t nb, double gam, double cfl, double mu,
                                                   int viscous, const T *__restrict__ W, const int32_t *__restrict__ ptr,
                                                   const int32_t *__restrict__ item, const double *__restrict__ S,
                                                   const double *__restrict__ A, const double *__restrict__ bA,
                                                   const double *__restrict__ V, T *__restrict__ dt)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / RG;
    const int g = (int)(t % RG);
    if (i >= n) return;  // whole row groups leave together
    const double rho = double(W[i]), ir = 1.0 / rho;
    const double u = double(W[n + i]) * ir, v = double(W[2 * n + i]) * ir, w = double(W[3 * n + i]) * ir;
    const double p = (gam - 1.0) * (double(W[4 * n + i]) - 0.5 * rho * (u * u + v * v + w * w));
    const double cs = sqrt(gam * p * ir);
    const double Vi = V[i];
    double sum = 0.0;
    for (int k = ptr[i] + g; k < ptr[i + 1]; k += RG) {
        const int it = item[k];
        double ax, ay, az, s;
        if (it >= 0) {
            const int j = it >> 1;
            ax = A[j];
            ay = A[m + j];
            az = A[2 * m + j];
            s = S[j];
        } else {
            const int q = -it - 1;
            ax = bA[q];
            ay = bA[nb + q];
            az = bA[2 * nb + q];
            s = sqrt(ax * ax + ay * ay + az * az);
        }
        const double uA = fabs(u * ax + v * ay + w * az);
        const double lam = cs + (viscous ? 2.0 * mu * s / (rho * Vi) : 0.0);
        sum += uA + lam * s;
    }
    sum = row_sum(sum);
    if (g == 0) dt[i] = T(cfl * Vi / sum);
}

template <class T>
__global__ void k_coarse_forcing(int64_t n5, const T *__restrict__ Rs, const T *__restrict__ R0, T *__restrict__ F)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n5) F[i] = Rs[i] - R0[i];
}

template <class T>
__global__ void k_coarse_update(int64_t n, const T *__restrict__ dt, const double *__restrict__ V,
                                const T *__restrict__ R, const T *__restrict__ F, T *__restrict__ W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T h = dt[i] / T(V[i]);
#pragma unroll
    for (int q = 0; q < 5; ++q) W[q * n + i] += h * (R[q * n + i] + F[q * n + i]);
}

template <class T>
__global__ void k_add(int64_t n5, const T *__restrict__ a, T *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n5) b[i] += a[i];
}

// restriction: Wc = sum V W / Vc (fine ids ascending), Rc = sum R; Tf fine type, Tc coarse type
template <class Tf, class Tc>
__global__ __launch_bounds__(256) void k_restrict(int64_t nc, int64_t nf, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ idx, const double *__restrict__ Vf,
                                                  const double *__restrict__ Vc, const Tf *__restrict__ Wf,
                                                  const Tf *__restrict__ Rf, Tc *__restrict__ Wc, Tc *__restrict__ Rc)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t k = t / RG;
    const int g = (int)(t % RG);
    if (k >= nc) return;  // whole row groups leave together
    const double vk = (g == 0 && Wc) ? Vc[k] : 1.0;  // requested ahead of the member loop
    double w[5] = {0, 0, 0, 0, 0}, r[5] = {0, 0, 0, 0, 0};
    for (int q = ptr[k] + g; q < ptr[k + 1]; q += RG) {
        const int i = idx[q];
        const double v = Vf[i];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            if (Wf) w[c] += v * double(Wf[c * nf + i]);
            if (Rf) r[c] += double(Rf[c * nf + i]);
        }
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        w[c] = row_sum(w[c]);
        r[c] = row_sum(r[c]);
    }
    if (g == 0)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            if (Wc) Wc[c * nc + k] = Tc(w[c] / vk);
            if (Rc) Rc[c * nc + k] = Tc(r[c]);
        }
}

template <class Tc, class Tf>
__global__ void k_prolong(int64_t nf, int64_t nc, const int32_t *__restrict__ f2c, const Tc *__restrict__ Wc,
                          const Tc *__restrict__ Wc0, Tf *__restrict__ Wf)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nf) return;
    const int k = f2c[i];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        if (Wc0) Wf[c * nf + i] += Tf(Wc[c * nc + k] - Wc0[c * nc + k]);
        else Wf[c * nf + i] += Tf(Wc[c * nc + k]);
    }
}

static Level *level_of(cgks_ctx *c, int level)
{
    if (level < 1 || level >= (int)c->lev.size()) throw Error{CGKS_E_STATE, "no such level: call cgks_agglomerate"};
    return c->lev[level];
}

// R = KFVS residual of W (+ add when given)
template <class T> static CoarseArgs<T> coarse_args(cgks_ctx *c, int level, const T *W, T *ff)
{
    Level *L = level_of(c, level);
    CoarseArgs<T> A;
    A.n = L->n;
    A.m = L->m;
    A.nb = L->nb;
    A.gam = c->prm.gamma;
    A.K = (5.0 - 3.0 * c->prm.gamma) / (c->prm.gamma - 1.0);
    A.W = W;
    A.pa = L->pa.p;
    A.pb = L->pb.p;
    A.bown = L->bown.p;
    A.btag = L->btag.p;
    A.A = L->A.p;
    A.bA = L->bA.p;
    A.bc = c->bc.p;
    A.fflux = ff;
    return A;
}

template <class T> static void kfvs_impl(cgks_ctx *c, int level, const T *W, T *R, T *ff, const T *add = nullptr)
{
    Level *L = level_of(c, level);
    CoarseArgs<T> A;
    A.n = L->n;
    A.m = L->m;
    A.nb = L->nb;
    A.gam = c->prm.gamma;
    A.K = (5.0 - 3.0 * c->prm.gamma) / (c->prm.gamma - 1.0);
    A.W = W;
    A.pa = L->pa.p;
    A.pb = L->pb.p;
    A.bown = L->bown.p;
    A.btag = L->btag.p;
    A.A = L->A.p;
    A.bA = L->bA.p;
    A.bc = c->bc.p;
    A.fflux = ff;
    const int64_t tot = L->m + L->nb;
    hipLaunchKernelGGL((k_kfvs_face<T>), G1(tot), dim3(256), 0, c->stream, A, (const T *)nullptr);
    hipLaunchKernelGGL((k_kfvs_gather<T>), GR(L->n), dim3(256), 0, c->stream, L->n, L->m, L->cf_ptr.p,
                       L->cf_item.p, ff, add, R);
}

void kfvs_residual(cgks_ctx *c, int level, const double *W, double *R)
{
    kfvs_impl<double>(c, level, W, R, level_of(c, level)->fflux.p);
}

void kfvs_residual32(cgks_ctx *c, int level, const float *W, float *R)
{
    Level *L = level_of(c, level);
    L->ffluxf.ensure(5 * (L->m + L->nb) + 5);
    kfvs_impl<float>(c, level, W, R, L->ffluxf.p);
}

template <class A, class B> __global__ void k_convert(int64_t n, const A *__restrict__ a, B *__restrict__ b)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = B(a[i]);
}

// FP32 KFVS residual of an FP64 state, returned in FP64 (the mixed-precision coarse operator)
void kfvs_residual_fp32(cgks_ctx *c, int level, const double *W, double *R)
{
    Level *L = level_of(c, level);
    const int64_t n5 = 5 * L->n;
    L->Wf.ensure(n5);
    L->Rf.ensure(n5);
    hipLaunchKernelGGL((k_convert<double, float>), G1(n5), dim3(256), 0, c->stream, n5, W, L->Wf.p);
    kfvs_residual32(c, level, L->Wf.p, L->Rf.p);
    hipLaunchKernelGGL((k_convert<float, double>), G1(n5), dim3(256), 0, c->stream, n5, L->Rf.p, R);
}

template <class T> static void coarse_dt_impl(cgks_ctx *c, int level, const T *W, T *dt, double cfl = -1.0)
{
    Level *L = level_of(c, level);
    hipLaunchKernelGGL((k_coarse_dt<T>), GR(L->n), dim3(256), 0, c->stream, L->n, L->m, L->nb, c->prm.gamma,
                       cfl > 0.0 ? cfl : c->prm.cfl, c->prm.mu, c->prm.viscous, W, L->cf_ptr.p, L->cf_item.p, L->S.p,
                       L->A.p, L->bA.p, L->V.p, dt);
}

void coarse_dt_level(cgks_ctx *c, int level, const double *W, double *dt) { coarse_dt_impl<double>(c, level, W, dt); }

static const double *finer_vol(cgks_ctx *c, int level)
{
    return level == 1 ? c->vol.p : c->lev[level - 1]->V.p;
}

void restrict_level(cgks_ctx *c, int level, const double *Wf, const double *Rf, double *Wc, double *Rc)
{
    Level *L = level_of(c, level);
    hipLaunchKernelGGL((k_restrict<double, double>), GR(L->n), dim3(256), 0, c->stream, L->n, L->nfine, L->c2f_ptr.p,
                       L->c2f_idx.p, finer_vol(c, level), L->V.p, Wf, Rf, Wc, Rc);
}

void prolong_level(cgks_ctx *c, int level, const double *dWc, double *Wf)
{
    Level *L = level_of(c, level);
    hipLaunchKernelGGL((k_prolong<double, double>), G1(L->nfine), dim3(256), 0, c->stream, L->nfine, L->n, L->f2c.p,
                       dWc, (const double *)nullptr, Wf);
}

// ---------------------------------------------------------------- implicit coarse smoother
// Backward Euler on a coarse level (paper Sec. 4.3), linearised with the Jacobian of a
// first-order Lax-Friedrichs flux, A+- = (A +- lambda I)/2, lambda = max(lambda_i, lambda_p),
// lambda = |U.n| + c + 2 mu S/(rho |Omega|).  The outward area vectors of a closed cell sum to
// zero, so the diagonal is |Omega_i|/dt_i + sum_p lambda_p S_p / 2; the neighbour products are
// formed without a matrix as F-(U_p + dU_p) - F-(U_p), F- = (F_n - lambda U)/2 with F_n the Euler
// flux along cell i's outward normal.  The system is solved by point relaxation: dU = rhs/D, then
// each sweep recomputes every cell from the previous sweep's neighbour increments (Jacobi order,
// so every cell of a sweep is independent and the result does not depend on the schedule).
// S is the coarse face's |A|, the factor of its KFVS flux.  A boundary face adds lambda S/2 with
// lambda the larger radius of owner and ghost state; its ghost increment is zero.
// One row of the cell -> face list per RG lanes, as in the KFVS gather.
template <class T> __device__ __forceinline__ void euler_flux_n(const T U[5], const double n[3], double gam, T F[5])
{
    const T ir = T(1) / U[0];
    const T un = (U[1] * T(n[0]) + U[2] * T(n[1]) + U[3] * T(n[2])) * ir;
    const T pr = T(gam - 1.0) * (U[4] - T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir);
    F[0] = U[0] * un;
#pragma unroll
    for (int d = 0; d < 3; ++d) F[1 + d] = U[1 + d] * un + pr * T(n[d]);
    F[4] = (U[4] + pr) * un;
}

template <class T>
__device__ __forceinline__ T spec_radius(const T U[5], const double n[3], double S, double V, double gam, double mu,
                                         int viscous)
{
    const T ir = T(1) / U[0];
    const T un = (U[1] * T(n[0]) + U[2] * T(n[1]) + U[3] * T(n[2])) * ir;
    const T pr = T(gam - 1.0) * (U[4] - T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir);
    const T c = Fp<T>::sqrt_(T(gam) * pr * ir);
    return abs_(un) + c + (viscous ? T(2.0 * mu * S / V) * ir : T(0));
}

template <class T> struct ImpArgs {
    int64_t n, m, nb;
    double gam, mu;
    int viscous;
    const T *W, *rhs, *dt;
    const int32_t *ptr, *item, *pa, *pb, *btag;
    const double *A, *bA, *V;  // pair area vectors [3][m], boundary area vectors [3][nb], volumes
    const BcTable *bc;
    T *lamS;       // per cell-face entry: lambda S / 2 (0 for a face of zero area)
    T *dg;         // diagonal per cell
    const T *din;  // previous iterate (sweeps)
    T *dout;       // increment written, or added when acc = 1
    int acc;
};

template <class T> __device__ __forceinline__ void load5(const T *W, int64_t n, int64_t i, T u[5])
{
#pragma unroll
    for (int q = 0; q < 5; ++q) u[q] = W[q * n + i];
}

// Diagonal, lambda S / 2 per entry and the first iterate dU = rhs / D.
template <class T> __global__ __launch_bounds__(256) void k_imp_diag(ImpArgs<T> a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / RG;
    const int g = (int)(t % RG);
    if (i >= a.n) return;  // whole row groups leave together
    const int64_t n = a.n;
    T Ui[5];
    load5(a.W, n, i, Ui);
    const double Vi = a.V[i];
    // the row's own epilogue inputs, requested before the face loop so their latency overlaps it
    T dti = T(1), rh[5], d0[5];
    if (g == 0) {
        dti = a.dt[i];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            rh[q] = a.rhs[q * n + i];
            d0[q] = a.acc ? a.dout[q * n + i] : T(0);
        }
    }
    T sum = T(0);
    for (int k = a.ptr[i] + g; k < a.ptr[i + 1]; k += RG) {
        const int it = a.item[k];
        double av[3];
        if (it >= 0) {
            const int j = it >> 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) av[d] = a.A[d * a.m + j];
        } else {
            const int q = -it - 1;
#pragma unroll
            for (int d = 0; d < 3; ++d) av[d] = a.bA[d * a.nb + q];
        }
        const double S = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
        T h = T(0);
        if (S > 0.0) {
            const double nv[3] = {av[0] / S, av[1] / S, av[2] / S};
            T Up[5];
            double Vp = Vi;
            if (it >= 0) {
                const int j = it >> 1;
                const int p = (it & 1) ? a.pa[j] : a.pb[j];
                load5(a.W, n, p, Up);
                Vp = a.V[p];
            } else {
                ghost_state(*a.bc, a.btag[-it - 1], nv, Ui, a.gam, Up);
            }
            const T li = spec_radius(Ui, nv, S, Vi, a.gam, a.mu, a.viscous);
            const T lp = spec_radius(Up, nv, S, Vp, a.gam, a.mu, a.viscous);
            h = T(0.5) * (li > lp ? li : lp) * T(S);
        }
        a.lamS[k] = h;
        sum += h;
    }
    sum = row_sum(sum);
    if (g == 0) {
        const T d = T(Vi) / dti + sum;
        a.dg[i] = d;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T v = rh[q] / d;
            a.dout[q * n + i] = a.acc ? d0[q] + v : v;
        }
    }
}

// One point-relaxation sweep: dU_i = (rhs_i - sum_p [F-(U_p + dU_p) - F-(U_p)] S_p) / D_i.
template <class T> __global__ __launch_bounds__(256) void k_imp_sweep(ImpArgs<T> a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = t / RG;
    const int g = (int)(t % RG);
    if (i >= a.n) return;  // whole row groups leave together
    const int64_t n = a.n;
    // the row's own epilogue inputs, requested before the face loop so their latency overlaps it
    T dgi = T(1), rh[5], d0[5];
    if (g == 0) {
        dgi = a.dg[i];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            rh[q] = a.rhs[q * n + i];
            d0[q] = a.acc ? a.dout[q * n + i] : T(0);
        }
    }
    T r[5] = {T(0), T(0), T(0), T(0), T(0)};
    for (int k = a.ptr[i] + g; k < a.ptr[i + 1]; k += RG) {
        const int it = a.item[k];
        if (it < 0) continue;  // boundary: zero ghost increment
        const T h = a.lamS[k];
        if (h == T(0)) continue;  // face of zero area
        const int j = it >> 1;
        const int p = (it & 1) ? a.pa[j] : a.pb[j];
        const double sg = (it & 1) ? -1.0 : 1.0;  // outward normal of cell i
        double av[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) av[d] = a.A[d * a.m + j];
        const double S = sqrt(av[0] * av[0] + av[1] * av[1] + av[2] * av[2]);
        const double nv[3] = {sg * av[0] / S, sg * av[1] / S, sg * av[2] / S};
        T Up[5], dp[5], Un[5], F1[5], F0[5];
        load5(a.W, n, p, Up);
        load5(a.din, n, p, dp);
#pragma unroll
        for (int q = 0; q < 5; ++q) Un[q] = Up[q] + dp[q];
        euler_flux_n(Un, nv, a.gam, F1);
        euler_flux_n(Up, nv, a.gam, F0);
        const T hS = T(0.5 * S);
#pragma unroll
        for (int q = 0; q < 5; ++q) r[q] += hS * (F1[q] - F0[q]) - h * dp[q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) r[q] = row_sum(r[q]);
    if (g == 0) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const T v = (rh[q] - r[q]) / dgi;
            a.dout[q * n + i] = a.acc ? d0[q] + v : v;
        }
    }
}

template <class T> struct ImpBufs {
    T *lamS, *dg, *dUa, *dUb, *dt;
};
template <class T> static ImpBufs<T> imp_bufs(Level *L);
template <> ImpBufs<double> imp_bufs<double>(Level *L)
{
    L->lamS.ensure(L->nnz + 1);
    L->dg.ensure(L->n);
    L->dUa.ensure(5 * L->n);
    L->dUb.ensure(5 * L->n);
    L->dt.ensure(L->n);
    return {L->lamS.p, L->dg.p, L->dUa.p, L->dUb.p, L->dt.p};
}
template <> ImpBufs<float> imp_bufs<float>(Level *L)
{
    L->lamSf.ensure(L->nnz + 1);
    L->dgf.ensure(L->n);
    L->dUaf.ensure(5 * L->n);
    L->dUbf.ensure(5 * L->n);
    L->dtf.ensure(L->n);
    return {L->lamSf.p, L->dgf.p, L->dUaf.p, L->dUbf.p, L->dtf.p};
}

// out = dU (acc = false) or out += dU (acc = true), dU the implicit increment at state W for rhs.
template <class T> static void implicit_solve(cgks_ctx *c, int l, const T *W, const T *rhs, T *out, bool acc)
{
    Level *L = level_of(c, l);
    ImpBufs<T> b = imp_bufs<T>(L);
    coarse_dt_impl<T>(c, l, W, b.dt, c->prm.cfl_implicit);
    ImpArgs<T> a;
    a.n = L->n;
    a.m = L->m;
    a.nb = L->nb;
    a.gam = c->prm.gamma;
    a.mu = c->prm.mu;
    a.viscous = c->prm.viscous;
    a.W = W;
    a.rhs = rhs;
    a.dt = b.dt;
    a.ptr = L->cf_ptr.p;
    a.item = L->cf_item.p;
    a.pa = L->pa.p;
    a.pb = L->pb.p;
    a.btag = L->btag.p;
    a.A = L->A.p;
    a.bA = L->bA.p;
    a.V = L->V.p;
    a.bc = c->bc.p;
    a.lamS = b.lamS;
    a.dg = b.dg;
    const int sweeps = c->prm.relax_sweeps;
    T *cur = b.dUa, *nxt = b.dUb;
    a.din = nullptr;
    a.dout = sweeps == 0 ? out : cur;
    a.acc = sweeps == 0 && acc;
    hipLaunchKernelGGL((k_imp_diag<T>), GR(L->n), dim3(256), 0, c->stream, a);
    for (int s = 1; s <= sweeps; ++s) {
        a.din = cur;
        a.dout = s == sweeps ? out : nxt;
        a.acc = s == sweeps && acc;
        hipLaunchKernelGGL((k_imp_sweep<T>), GR(L->n), dim3(256), 0, c->stream, a);
        std::swap(cur, nxt);
    }
}

void coarse_implicit(cgks_ctx *c, int level, const double *W, const double *rhs, double *dU)
{
    implicit_solve<double>(c, level, W, rhs, dU, false);
}

// FP32 implicit increment of FP64 inputs, returned in FP64 (the mixed-precision coarse smoother)
void coarse_implicit_fp32(cgks_ctx *c, int level, const double *W, const double *rhs, double *dU)
{
    Level *L = level_of(c, level);
    const int64_t n5 = 5 * L->n;
    L->Wf.ensure(n5);
    L->Rf.ensure(n5);
    L->Df.ensure(n5);
    hipLaunchKernelGGL((k_convert<double, float>), G1(n5), dim3(256), 0, c->stream, n5, W, L->Wf.p);
    hipLaunchKernelGGL((k_convert<double, float>), G1(n5), dim3(256), 0, c->stream, n5, rhs, L->Rf.p);
    implicit_solve<float>(c, level, L->Wf.p, L->Rf.p, L->Df.p, false);
    hipLaunchKernelGGL((k_convert<float, double>), G1(n5), dim3(256), 0, c->stream, n5, L->Df.p, dU);
}

// ---------------------------------------------------------------- V-cycle (FP64 and mixed)
// Coarse levels work in delta form: each level keeps its restricted state W0 and
// the correction D = W - W0.  Because Res_2h(W0) + F = Res*_2h, the first sweep
// is D = dt/V Res* exactly; the correction therefore vanishes with the fine
// residual in any precision, and no bits of W0 are lost when it is prolonged.
template <class T>
__global__ void k_delta_update(int64_t n, const T *__restrict__ dt, const double *__restrict__ V, const T *__restrict__ R,
                               const T *__restrict__ F, T *__restrict__ D)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const T h = dt[i] / T(V[i]);
#pragma unroll
    for (int q = 0; q < 5; ++q) D[q * n + i] += h * (R[q * n + i] + F[q * n + i]);
}

template <class T>
__global__ void k_sum_state(int64_t n5, const T *__restrict__ W0, const T *__restrict__ D, T *__restrict__ W)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n5) W[i] = W0[i] + D[i];
}

template <class T> struct LevelBufs {
    T *W0, *W, *D, *R, *F, *Rs, *dt, *ff;
};

template <class T> static LevelBufs<T> bufs(Level *L);
template <> LevelBufs<double> bufs<double>(Level *L)
{
    L->D.ensure(5 * L->n);
    return {L->W0.p, L->W.p, L->D.p, L->R.p, L->F.p, L->Rs.p, L->dt.p, L->fflux.p};
}
template <> LevelBufs<float> bufs<float>(Level *L)
{
    const size_t n5 = 5 * L->n;
    L->W0f.ensure(n5);
    L->Wf.ensure(n5);
    L->Df.ensure(n5);
    L->Rf.ensure(n5);
    L->Ff.ensure(n5);
    L->Rsf.ensure(n5);
    L->dtf.ensure(L->n);
    L->ffluxf.ensure(5 * (L->m + L->nb) + 5);
    return {L->W0f.p, L->Wf.p, L->Df.p, L->Rf.p, L->Ff.p, L->Rsf.p, L->dtf.p, L->ffluxf.p};
}

// A coarse sweep at W = W0 + D: forward Euler D += dt/V (Res_2h(W) + F), or D += dU of the
// implicit smoother with right-hand side Res_2h(W) + F.
template <class T> static void coarse_sweep(cgks_ctx *c, int l)
{
    Level *L = c->lev[l];
    LevelBufs<T> b = bufs<T>(L);
    hipStream_t st = c->stream;
    const int64_t n = L->n, n5 = 5 * n;
    hipLaunchKernelGGL((k_sum_state<T>), G1(n5), dim3(256), 0, st, n5, b.W0, b.D, b.W);
    if (c->prm.coarse_smoother == 1) {
        kfvs_impl<T>(c, l, b.W, b.R, b.ff, b.F);
        implicit_solve<T>(c, l, b.W, b.R, b.D, true);
    } else {
        kfvs_impl<T>(c, l, b.W, b.R, b.ff);
        coarse_dt_impl<T>(c, l, b.W, b.dt);
        hipLaunchKernelGGL((k_delta_update<T>), G1(n), dim3(256), 0, st, n, b.dt, L->V.p, b.R, b.F, b.D);
    }
}

template <class T> static void coarse_visit(cgks_ctx *c, int l);

// One FAS cycle on level l (>= 1) with its forcing F and correction D set: the pre-sweeps not
// yet applied, then (above the coarsest level) a visit of level l + 1 from the restricted state
// and residual, the prolonged correction, and the post-sweeps.
template <class T> static void fas_level(cgks_ctx *c, int l, int pre_done)
{
    Level *L = c->lev[l];
    LevelBufs<T> b = bufs<T>(L);
    hipStream_t st = c->stream;
    for (int s = pre_done; s < c->prm.nu_pre[l]; ++s) coarse_sweep<T>(c, l);
    if (l + 1 < (int)c->lev.size()) {
        Level *C = c->lev[l + 1];
        LevelBufs<T> cb = bufs<T>(C);
        // fluxes at W0 + D, then W = W0 + D and Res_2h(W) + F in the gather
        const CoarseArgs<T> ca = coarse_args<T>(c, l, b.W0, b.ff);
        hipLaunchKernelGGL((k_kfvs_face<T>), G1(L->m + L->nb), dim3(256), 0, st, ca, (const T *)b.D);
        hipLaunchKernelGGL((k_kfvs_rows<T, false>), GR(L->n), dim3(256), 0, st, ca, (const T *)b.ff, L->cf_ptr.p,
                           L->cf_item.p, L->AS.p, L->V.p, 0.0, 0.0, 0, (const T *)nullptr, (const T *)b.D, b.F,
                           (T *)nullptr, b.W, b.R);
        hipLaunchKernelGGL((k_restrict<T, T>), GR(C->n), dim3(256), 0, st, C->n, C->nfine, C->c2f_ptr.p, C->c2f_idx.p,
                           L->V.p, C->V.p, b.W, b.R, cb.W0, cb.Rs);
        coarse_visit<T>(c, l + 1);
        hipLaunchKernelGGL((k_prolong<T, T>), G1(C->nfine), dim3(256), 0, st, C->nfine, C->n, C->f2c.p, cb.D,
                           (const T *)nullptr, b.D);
    }
    for (int s = 0; s < c->prm.nu_post[l]; ++s) coarse_sweep<T>(c, l);
}

// Visit of level l (>= 1) from its parent, with W0 and Rs set: forcing F = Res* - Res_2h(W0),
// then cycle_gamma FAS cycles (1: V-cycle, 2: W-cycle), each continuing from W0 + D with the
// same forcing; leaves the correction in D.
template <class T> static void coarse_visit(cgks_ctx *c, int l)
{
    Level *L = c->lev[l];
    LevelBufs<T> b = bufs<T>(L);
    hipStream_t st = c->stream;
    const int64_t n = L->n, n5 = 5 * n;
    const int npre = c->prm.nu_pre[l];
    const bool implicit = c->prm.coarse_smoother == 1;
    // the first sweep at W = W0 has right-hand side Res_2h(W0) + F = Res* exactly
    if (npre > 0 && !implicit) {
        // face fluxes at W0, then the gather with the local step, forcing and first sweep
        const CoarseArgs<T> ca = coarse_args<T>(c, l, b.W0, b.ff);
        hipLaunchKernelGGL((k_kfvs_face<T>), G1(L->m + L->nb), dim3(256), 0, st, ca, (const T *)nullptr);
        hipLaunchKernelGGL((k_kfvs_rows<T, true>), GR(n), dim3(256), 0, st, ca, (const T *)b.ff, L->cf_ptr.p,
                           L->cf_item.p, L->AS.p, L->V.p, c->prm.cfl, c->prm.mu, c->prm.viscous, (const T *)b.Rs,
                           (const T *)nullptr, b.F, b.D, (T *)nullptr, (T *)nullptr);
    } else {
        kfvs_impl<T>(c, l, b.W0, b.R, b.ff);
        hipLaunchKernelGGL((k_coarse_forcing<T>), G1(n5), dim3(256), 0, st, n5, b.Rs, b.R, b.F);
        if (npre > 0) implicit_solve<T>(c, l, b.W0, b.Rs, b.D, false);
        else CGKS_HIP(hipMemsetAsync(b.D, 0, sizeof(T) * n5, st));
    }
    const int gamma = std::max(1, c->prm.cycle_gamma);
    for (int k = 0; k < gamma; ++k) fas_level<T>(c, l, k == 0 && npre > 0 ? 1 : 0);
}

// One V-cycle on the fine state; the norm of the smoothing residual is left in c->scal[0].
void vcycle_once(cgks_ctx *c, double *W, double *G, double *alpha, bool fp32_flux, bool fp32_coarse,
                 double *norm_out)
{
    hipStream_t st = c->stream;
    const int nb = gather_blocks(c->N);
    c->partial.ensure(nb);
    const int npre = std::max(1, c->prm.nu_pre[0]);
    float *c32 = fp32_flux ? c->coeff.p : nullptr;  // FP32 coefficients in the FP32 flux phase
    for (int s = 0; s < npre; ++s) {
        launch_local_dt_recon(c, W, G, alpha, c->dtc.p, c->coef.p, nullptr, c32);
        launch_face(c, MODE_RES, c->coef.p, c->dtc.p, -1.0, fp32_flux);
        launch_gather_fe(c, W, G, alpha, c->dtc.p, c->Rw.p, s == 0 ? c->partial.p : nullptr);
        if (s == 0) finish_norm(c, c->partial.p, nb, c->N, norm_out);
    }
    if (c->lev.size() > 1) {
        launch_local_dt_recon(c, W, G, alpha, c->dtc.p, c->coef.p, nullptr, c32);
        launch_face(c, MODE_RESONLY, c->coef.p, c->dtc.p, -1.0, fp32_flux);
        launch_gather_res(c, c->Rw.p, nullptr, nullptr, MODE_RESONLY);
        Level *L = c->lev[1];
        if (!fp32_coarse) {
            LevelBufs<double> b = bufs<double>(L);
            hipLaunchKernelGGL((k_restrict<double, double>), GR(L->n), dim3(256), 0, st, L->n, L->nfine, L->c2f_ptr.p,
                               L->c2f_idx.p, c->vol.p, L->V.p, W, c->Rw.p, b.W0, b.Rs);
            coarse_visit<double>(c, 1);
            hipLaunchKernelGGL((k_prolong<double, double>), G1(L->nfine), dim3(256), 0, st, L->nfine, L->n, L->f2c.p,
                               b.D, (const double *)nullptr, W);
        } else {
            LevelBufs<float> b = bufs<float>(L);
            hipLaunchKernelGGL((k_restrict<double, float>), GR(L->n), dim3(256), 0, st, L->n, L->nfine, L->c2f_ptr.p,
                               L->c2f_idx.p, c->vol.p, L->V.p, W, c->Rw.p, b.W0, b.Rs);
            coarse_visit<float>(c, 1);
            hipLaunchKernelGGL((k_prolong<float, double>), G1(L->nfine), dim3(256), 0, st, L->nfine, L->n, L->f2c.p,
                               b.D, (const float *)nullptr, W);
        }
    }
    for (int s = 0; s < c->prm.nu_post[0]; ++s) {
        launch_local_dt_recon(c, W, G, alpha, c->dtc.p, c->coef.p, nullptr, c32);
        launch_face(c, MODE_RES, c->coef.p, c->dtc.p, -1.0, fp32_flux);
        launch_gather_fe(c, W, G, alpha, c->dtc.p, c->Rw.p, nullptr);
    }
}

}  // namespace cgks

// C ABI entry points of libcgks (see include/cgks.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <parallel/algorithm>

#include "common.hpp"

using namespace cgks;

cgks_ctx::~cgks_ctx()
{
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
    for (Level *l : lev) delete l;
    lev.clear();
    if (pinned) (void)hipHostFree(pinned);
    if (pinned_i) (void)hipHostFree(pinned_i);
    delete adj;
}

#define API_BEGIN(ctx)                                     \
    if (!(ctx)) return CGKS_E_ARG;                         \
    try {
#define API_END(ctx)                                       \
    }                                                      \
    catch (const cgks::Error &e)                           \
    {                                                      \
        (ctx)->err = e.msg;                                \
        return e.code;                                     \
    }                                                      \
    catch (const std::exception &e)                        \
    {                                                      \
        (ctx)->err = e.what();                             \
        return CGKS_E_DEVICE;                              \
    }                                                      \
    return CGKS_OK;

static void need_mesh(const cgks_ctx *c)
{
    if (!c->has_mesh) throw Error{CGKS_E_STATE, "no mesh: call cgks_set_mesh first"};
}

// evaluations that reach boundary faces need a condition for every tag the mesh uses
static void need_bc(const cgks_ctx *c)
{
    need_mesh(c);
    const uint64_t missing = c->tags_used & ~c->tags_set;
    if (missing) {
        int t = 0;
        while (!((missing >> t) & 1)) ++t;
        throw Error{CGKS_E_STATE, "boundary tag " + std::to_string(t) + " has no boundary condition: call cgks_set_bc"};
    }
}

static void check_params(const cgks_params *p)
{
    if (!(p->gamma > 1.0 && p->gamma < 5.0 / 3.0 + 1e-12)) throw Error{CGKS_E_ARG, "gamma must be in (1, 5/3]"};
    if (!(p->cfl > 0.0)) throw Error{CGKS_E_ARG, "cfl must be positive"};
    if (p->viscous && !(p->mu > 0.0)) throw Error{CGKS_E_ARG, "viscous flow needs mu > 0"};
    if (!(p->prandtl > 0.0)) throw Error{CGKS_E_ARG, "prandtl must be positive"};
    if (!(p->gamma_lin > 0.0 && p->gamma_lin < 1.0)) throw Error{CGKS_E_ARG, "gamma_lin must be in (0,1)"};
    if (p->levels < 1 || p->levels > 8) throw Error{CGKS_E_ARG, "levels must be in 1..8"};
    if (p->passes < 0 || p->passes > 16) throw Error{CGKS_E_ARG, "passes must be in 0..16"};
    if (p->precision != 0 && p->precision != 1) throw Error{CGKS_E_ARG, "precision must be 0 or 1"};
    if (p->coarse_smoother != 0 && p->coarse_smoother != 1) throw Error{CGKS_E_ARG, "coarse_smoother must be 0 or 1"};
    if (p->relax_sweeps < 0 || p->relax_sweeps > 64) throw Error{CGKS_E_ARG, "relax_sweeps must be in 0..64"};
    if (p->coarse_smoother == 1 && !(p->cfl_implicit > 0.0)) throw Error{CGKS_E_ARG, "cfl_implicit must be positive"};
    if (p->cycle_gamma < 1 || p->cycle_gamma > 3) throw Error{CGKS_E_ARG, "cycle_gamma must be in 1..3"};
    if (p->cell_order < 0 || p->cell_order > 2) throw Error{CGKS_E_ARG, "cell_order must be 0, 1 or 2"};
    if (p->mixed_stall < 1) throw Error{CGKS_E_ARG, "mixed_stall must be at least 1"};
    if (p->adjoint_tape != 0 && p->adjoint_tape != 1) throw Error{CGKS_E_ARG, "adjoint_tape must be 0 or 1"};
}

static void check_bad(cgks_ctx *c)
{
    CGKS_HIP(hipMemcpyAsync(c->pinned_i, c->bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    CGKS_HIP(hipStreamSynchronize(c->stream));
    if (*c->pinned_i != INT32_MAX) {
        const int32_t cell = *c->pinned_i;
        const int32_t big = INT32_MAX;
        CGKS_HIP(hipMemcpyAsync(c->bad.p, &big, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
        CGKS_HIP(hipStreamSynchronize(c->stream));
        throw Error{CGKS_E_PHYS, "non-positive density or pressure at a Gauss point of cell " +
                                      std::to_string(c->caller_cell(cell))};
    }
}

// ---------------------------------------------------------------- internal cell order
// Cells are stored in a locality order (element type, then the Hilbert curve through the cell
// centroids): consecutive cells,
// and so the faces sorted by them, are close in space, which keeps the neighbour gathers of the
// reconstruction, face and gather kernels within a few cache lines whatever order the caller's
// mesh generator emitted.  Cell arrays at the ABI are moved between the caller's order and this
// one by the two kernels below (component c of cell i: c N + i).
__global__ void k_cells_in(int64_t N, const int32_t *__restrict__ perm, const double *__restrict__ src,
                           double *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t c = blockIdx.y;
    dst[c * N + i] = src[c * N + perm[i]];
}

template <class T>
__global__ void k_cells_out(int64_t N, const int32_t *__restrict__ perm, const T *__restrict__ src, T *__restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t c = blockIdx.y;
    dst[c * N + perm[i]] = src[c * N + i];
}

// arrays at the ABI are in the caller's order and must be moved
static bool io_moved(const cgks_ctx *c) { return c->permuted && c->prm.cell_order == 1; }

// caller-order input -> internal order in staging slot `slot` (or the caller's pointer itself)
static double *cells_in(cgks_ctx *c, const double *user, int ncomp, int slot)
{
    if (!user || !io_moved(c)) return const_cast<double *>(user);
    DBuf<double> &b = c->io[slot];
    b.ensure((size_t)ncomp * c->N);
    hipLaunchKernelGGL(k_cells_in, dim3(blocks_for(c->N, 256), ncomp), dim3(256), 0, c->stream, c->N, c->perm.p,
                       user, b.p);
    return b.p;
}

// where an output in the internal order is written before cells_out moves it to the caller
static double *cells_buf(cgks_ctx *c, double *user, int ncomp, int slot)
{
    if (!user || !io_moved(c)) return user;
    c->io[slot].ensure((size_t)ncomp * c->N);
    return c->io[slot].p;
}

template <class T> static void cells_scatter(cgks_ctx *c, const T *src, T *user, int ncomp)
{
    hipLaunchKernelGGL(k_cells_out<T>, dim3(blocks_for(c->N, 256), ncomp), dim3(256), 0, c->stream, c->N, c->perm.p,
                       src, user);
}

static void cells_out(cgks_ctx *c, double *user, int ncomp, int slot)
{
    if (!user || !io_moved(c)) return;
    cells_scatter(c, c->io[slot].p, user, ncomp);
}

// Hilbert index of a point with 21-bit coordinates q[3]: Skilling's transform of the axes into
// the "transposed" Hilbert index (J. Skilling, Programming the Hilbert curve, AIP Conf. Proc. 707,
// 2004), whose bits, interleaved, give the position along the curve.
static uint64_t hilbert_key(const uint32_t q[3])
{
    constexpr int B = 21;
    uint32_t X[3] = {q[0], q[1], q[2]};
    for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
        for (int d = 0; d < 3; ++d) {
            if (X[d] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[d]) & P;
                X[0] ^= t;
                X[d] ^= t;
            }
        }
    }
    for (int d = 1; d < 3; ++d) X[d] ^= X[d - 1];
    uint32_t t = 0;
    for (uint32_t Q = 1u << (B - 1); Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
    for (int d = 0; d < 3; ++d) X[d] ^= t;
    uint64_t key = 0;
    for (int b = B - 1; b >= 0; --b)
        for (int d = 0; d < 3; ++d) key = (key << 1) | ((X[d] >> b) & 1u);
    return key;
}

// Locality order of the cells: by element type, then along the Hilbert curve through the cell
// centroids (node means), ties by caller id.  Blocks of one element type keep the reconstruction's
// 64-cell groups uniform in their neighbour count and the face kernel's waves uniform in Gauss
// points per face; the curve keeps each cell's neighbours a few cache lines away.
static std::vector<int32_t> locality_order(int64_t N, int64_t n_nodes, const double *xyz, const uint8_t *ctype,
                                           const int64_t *cptr, const int64_t *cnode)
{
    std::vector<double> x(3 * N);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = 0; i < N; ++i) {
        const int t = ctype[i];
        if ((t != 4 && t != 5 && t != 6 && t != 8) || cptr[i + 1] - cptr[i] != t)
            throw Error{CGKS_E_MESH, "cell " + std::to_string(i) + ": unsupported type or node count"};
        double m[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < t; ++a) {
            const int64_t nd = cnode[cptr[i] + a];
            if (nd < 0 || nd >= n_nodes) throw Error{CGKS_E_MESH, "cell " + std::to_string(i) + ": node out of range"};
            for (int d = 0; d < 3; ++d) m[d] += xyz[3 * nd + d];
        }
        for (int d = 0; d < 3; ++d) {
            x[3 * i + d] = m[d] / t;
            lo[d] = std::min(lo[d], x[3 * i + d]);
            hi[d] = std::max(hi[d], x[3 * i + d]);
        }
    }
    std::vector<uint64_t> key(N);
    for (int64_t i = 0; i < N; ++i) {
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            const double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            const double u = (x[3 * i + d] - lo[d]) / span;
            q[d] = (uint32_t)std::min(2097151.0, std::max(0.0, u * 2097151.0));
        }
        key[i] = hilbert_key(q);
    }
    std::vector<int32_t> perm(N);
    for (int64_t i = 0; i < N; ++i) perm[i] = (int32_t)i;
    __gnu_parallel::sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
        if (ctype[a] != ctype[b]) return ctype[a] < ctype[b];
        return key[a] != key[b] ? key[a] < key[b] : a < b;
    });
    return perm;
}

// ---------------------------------------------------------------- work memory without allocation
// cgks_residual_noalloc takes its work memory (local steps, polynomial coefficients, boundary
// ghost states, face records and, with cell_order 1, the reordered inputs and outputs) from this
// file-scope device array instead of the context's buffers or hipMalloc.  Every GPU the library
// runs on holds its own copy until the process ends.  Host code never passes the array's name to
// a kernel: its device address is looked up once per device with hipGetSymbolAddress and kept.
static constexpr size_t SCRATCH_DOUBLES = size_t(32) << 20;  // 32 Mi doubles = 256 MiB
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[256];

static double *scratch_on_device(int device)
{
    if (device < 0 || device >= 256) throw Error{CGKS_E_DEVICE, "device ordinal out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error{CGKS_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch_ptr[device] = static_cast<double *>(ptr);
    }
    return g_scratch_ptr[device];
}

static cgks_status vcycle_impl(cgks_ctx *c, double *W, double *G, double *alpha, int32_t max_cycles,
                               double tol_drop, double *hist, int32_t *n_done)
{
    need_bc(c);
    if (!W || !G || !alpha || max_cycles < 0) throw Error{CGKS_E_ARG, "bad arguments"};
    if (c->prm.levels > 1 && (int)c->lev.size() != c->prm.levels) build_hierarchy(c);
    if (n_done) *n_done = 0;
    double r0 = 0.0, best = 0.0;
    int best_at = 0;
    bool mixed = c->prm.precision == 1;
    const int64_t N = c->N;
    // The loop's decisions after each cycle: record the norm, then stop (converged), switch the
    // mixed cycle to FP64, or go on.  Returns 1 to stop, 2 for a precision switch, 0 otherwise.
    auto decide = [&](int32_t k, double r) -> int {
        if (!std::isfinite(r)) throw Error{CGKS_E_NONFINITE, "non-finite residual in cycle " + std::to_string(k)};
        if (hist) hist[k] = r;
        if (n_done) *n_done = k + 1;
        if (k == 0) {
            r0 = r;
            best = r;
            if (r == 0.0) return 1;
        }
        if (r < best) best = r, best_at = k;
        const double drop = r / r0;
        if (drop <= tol_drop) return 1;
        if (mixed && (drop <= c->prm.mixed_switch || k - best_at >= c->prm.mixed_stall)) return 2;
        return 0;
    };
    // Cycles run in batches queued without a host wait, each cycle writing its norm into a
    // device history read once per batch.  The state at the start of a batch is kept; when the
    // history shows that the loop stops or switches precision before the batch's last cycle, the
    // state is restored and the batch re-run up to that cycle, and a non-physical state found at
    // the end of a batch is located by re-running the batch one cycle at a time.  The kernels are
    // deterministic, so results are those of a loop that reads every norm.  Without a tolerance
    // in FP64 one batch holds every cycle.
    const int32_t B = (tol_drop <= 0.0 && !mixed) ? std::min<int32_t>(max_cycles, 1 << 22) : 16;
    if (max_cycles > 0) c->hist_dev.ensure((size_t)B);
    auto save = [&](bool back) {
        const size_t n5 = 5 * N * sizeof(double), n15 = 15 * N * sizeof(double), n1 = N * sizeof(double);
        if (!back) {
            c->snapW.ensure(5 * N);
            c->snapG.ensure(15 * N);
            c->snapA.ensure(N);
        }
        CGKS_HIP(hipMemcpyAsync(back ? W : c->snapW.p, back ? c->snapW.p : W, n5, hipMemcpyDeviceToDevice, c->stream));
        CGKS_HIP(hipMemcpyAsync(back ? G : c->snapG.p, back ? c->snapG.p : G, n15, hipMemcpyDeviceToDevice, c->stream));
        CGKS_HIP(hipMemcpyAsync(back ? alpha : c->snapA.p, back ? c->snapA.p : alpha, n1, hipMemcpyDeviceToDevice,
                                c->stream));
    };
    int32_t k = 0;
    while (k < max_cycles) {
        const int32_t nb = std::min(B, max_cycles - k);
        const bool keep = nb > 1;
        if (keep) save(false);
        const bool mb = mixed;
        for (int32_t j = 0; j < nb; ++j) {
            vcycle_once(c, W, G, alpha, mb, mb, c->hist_dev.p + j);
            CGKS_HIP(hipGetLastError());
        }
        CGKS_HIP(hipMemcpyAsync(c->pinned_i, c->bad.p, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        const std::vector<double> h = c->hist_dev.download((size_t)nb, c->stream);
        if (*c->pinned_i != INT32_MAX) {
            if (!keep) check_bad(c);
            // re-run the batch from its start as the checked loop: a check after every cycle
            save(true);
            const int32_t clear = INT32_MAX;
            CGKS_HIP(hipMemcpyAsync(c->bad.p, &clear, sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
            for (int32_t j = 0; j < nb; ++j) {
                vcycle_once(c, W, G, alpha, mixed, mixed, c->hist_dev.p + j);
                CGKS_HIP(hipGetLastError());
                check_bad(c);
                CGKS_HIP(hipMemcpyAsync(c->pinned, c->hist_dev.p + j, sizeof(double), hipMemcpyDeviceToHost, c->stream));
                CGKS_HIP(hipStreamSynchronize(c->stream));
                const int what = decide(k + j, c->pinned[0]);
                if (what == 1) return CGKS_OK;
                if (what == 2) mixed = false;
            }
            k += nb;
            continue;
        }
        int32_t stop = -1, what = 0;
        for (int32_t j = 0; j < nb && stop < 0; ++j) {
            const double r = h[j];
            if (!std::isfinite(r) && j + 1 < nb) {
                // the state the checked loop would leave: after cycle k + j
                save(true);
                for (int32_t q = 0; q <= j; ++q) vcycle_once(c, W, G, alpha, mb, mb, c->hist_dev.p + q);
                CGKS_HIP(hipStreamSynchronize(c->stream));
            }
            what = decide(k + j, r);
            if (what) stop = j;
        }
        if (stop < 0) {
            k += nb;
            continue;
        }
        if (stop + 1 < nb) {
            save(true);
            for (int32_t q = 0; q <= stop; ++q) {
                vcycle_once(c, W, G, alpha, mb, mb, c->hist_dev.p + q);
                CGKS_HIP(hipGetLastError());
            }
        }
        if (what == 1) {
            CGKS_HIP(hipStreamSynchronize(c->stream));
            return CGKS_OK;
        }
        mixed = false;
        k += stop + 1;
    }
    CGKS_HIP(hipStreamSynchronize(c->stream));
    c->err = "residual drop not reached in max_cycles";
    return CGKS_E_NOCONV;
}



extern "C" {

cgks_status cgks_default_params(cgks_params *p)
{
    if (!p) return CGKS_E_ARG;
    std::memset(p, 0, sizeof(*p));
    p->gamma = 1.4;
    p->mu = 0.0;
    p->prandtl = 1.0;
    p->cfl = 0.5;
    p->eps_tau = 0.01;
    p->c_tau = 1.0;
    p->weno_eps = 1e-5;
    p->gamma_lin = 0.5;
    p->skew_delta = 0.25;
    p->skew_sin = 0.17364817766693033;  // sin 10 deg
    p->viscous = 0;
    p->levels = 3;
    p->passes = 3;
    p->precision = 0;
    for (int l = 0; l < 8; ++l) {
        p->nu_pre[l] = 1;
        p->nu_post[l] = 0;
    }
    p->mixed_switch = 1e-6;
    p->seed = 1;
    p->coarse_smoother = 0;
    p->relax_sweeps = 2;
    p->cfl_implicit = 0.25;
    p->cycle_gamma = 1;
    p->cell_order = 1;
    p->mixed_stall = 300;
    p->adjoint_tape = 0;
    return CGKS_OK;
}

cgks_status cgks_create(const cgks_params *p, cgks_ctx **out)
{
    if (!p || !out) return CGKS_E_ARG;
    cgks_ctx *c = new (std::nothrow) cgks_ctx();
    if (!c) return CGKS_E_DEVICE;
    try {
        check_params(p);
        c->prm = *p;
        CGKS_HIP(hipGetDevice(&c->device));
        hipDeviceProp_t prop;
        CGKS_HIP(hipGetDeviceProperties(&prop, c->device));
        c->gpu_cus = prop.multiProcessorCount;
        c->scratch = scratch_on_device(c->device);
        CGKS_HIP(hipHostMalloc((void **)&c->pinned, 64 * sizeof(double), hipHostMallocDefault));
        CGKS_HIP(hipHostMalloc((void **)&c->pinned_i, 16 * sizeof(int32_t), hipHostMallocDefault));
        for (int t = 0; t < 64; ++t) {
            c->bc_host.kind[t] = CGKS_BC_SLIP;
            for (int k = 0; k < 5; ++k) c->bc_host.prim[t][k] = 0.0;
        }
        c->bc.alloc(1);
        CGKS_HIP(hipMemcpy(c->bc.p, &c->bc_host, sizeof(BcTable), hipMemcpyHostToDevice));
        c->lev.push_back(nullptr);
    } catch (const Error &e) {
        int code = e.code;
        delete c;
        return (cgks_status)code;
    } catch (...) {
        delete c;
        return CGKS_E_DEVICE;
    }
    *out = c;
    return CGKS_OK;
}

void cgks_destroy(cgks_ctx *c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    delete c;
}

const char *cgks_last_error(const cgks_ctx *c) { return c ? c->err.c_str() : "null context"; }

cgks_status cgks_set_params(cgks_ctx *c, const cgks_params *p)
{
    API_BEGIN(c)
    if (c->adj) c->adj->ready = false;  // the linearisation no longer matches
    if (!p) throw Error{CGKS_E_ARG, "null params"};
    check_params(p);
    if (c->has_mesh && (p->cell_order == 0) != (c->prm.cell_order == 0))
        throw Error{CGKS_E_ARG, "cell_order 0 against 1/2 is fixed by cgks_set_mesh: set the mesh again"};
    const cgks_params prev = c->prm;
    c->prm = *p;
    if (c->prm.precision == 1) {
        try {
            ensure_fp32_front(c);
        } catch (...) {  // the previous parameters stay in force
            c->prm = prev;
            throw;
        }
    }
    API_END(c)
}

cgks_status cgks_set_stream(cgks_ctx *c, void *s)
{
    API_BEGIN(c)
    c->stream = (hipStream_t)s;
    API_END(c)
}

cgks_status cgks_set_mesh(cgks_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_cells, const uint8_t *ctype,
                          const int64_t *cnode_ptr, const int64_t *cnode, int64_t n_bfaces, const int64_t *bnode_ptr,
                          const int64_t *bnode, const int32_t *btag, const int64_t *node_canon)
{
    API_BEGIN(c)
    if (c->adj) c->adj->ready = false;  // the linearisation no longer matches
    if (!xyz || !ctype || !cnode_ptr || !cnode || (n_bfaces > 0 && (!bnode_ptr || !bnode || !btag)) || n_bfaces < 0)
        throw Error{CGKS_E_ARG, "null mesh array"};
    for (Level *l : c->lev) delete l;
    c->lev.assign(1, nullptr);
    c->has_mesh = false;
    c->opf.release();
    c->lgeof.release();
    c->coeff.release();
    c->permuted = false;
    c->perm_h.clear();
    if (n_cells <= 0 || n_nodes <= 0 || n_cells > INT32_MAX / 2 || n_nodes > INT32_MAX)
        throw Error{CGKS_E_ARG, "mesh sizes out of range"};
    if (c->prm.cell_order == 0) {
        mesh_build(c, n_nodes, xyz, n_cells, ctype, cnode_ptr, cnode, n_bfaces, bnode_ptr, bnode, btag, node_canon);
    } else {
        std::vector<int32_t> perm = locality_order(n_cells, n_nodes, xyz, ctype, cnode_ptr, cnode);
        std::vector<uint8_t> ct(n_cells);
        std::vector<int64_t> cp(n_cells + 1, 0), cn(cnode_ptr[n_cells]);
        for (int64_t i = 0; i < n_cells; ++i) {
            const int64_t o = perm[i];
            ct[i] = ctype[o];
            cp[i + 1] = cp[i] + (cnode_ptr[o + 1] - cnode_ptr[o]);
            std::copy(cnode + cnode_ptr[o], cnode + cnode_ptr[o + 1], cn.begin() + cp[i]);
        }
        c->perm_h = std::move(perm);
        c->permuted = true;
        mesh_build(c, n_nodes, xyz, n_cells, ct.data(), cp.data(), cn.data(), n_bfaces, bnode_ptr, bnode, btag,
                   node_canon);
    }
    c->perm.upload(c->permuted ? c->perm_h : std::vector<int32_t>(), c->stream);
    CGKS_HIP(hipStreamSynchronize(c->stream));
    // host copy of the mesh in the internal order (parameter sensitivities rebuild its geometry)
    {
        auto &H = c->hmesh;
        H.n_nodes = n_nodes;
        H.n_bf = n_bfaces;
        H.xyz.assign(xyz, xyz + 3 * n_nodes);
        H.ct.resize(n_cells);
        H.cp.assign(n_cells + 1, 0);
        H.cn.resize(cnode_ptr[n_cells]);
        for (int64_t i = 0; i < n_cells; ++i) {
            const int64_t o = c->caller_cell(i);
            H.ct[i] = ctype[o];
            H.cp[i + 1] = H.cp[i] + (cnode_ptr[o + 1] - cnode_ptr[o]);
            std::copy(cnode + cnode_ptr[o], cnode + cnode_ptr[o + 1], H.cn.begin() + H.cp[i]);
        }
        H.bp.assign(bnode_ptr ? bnode_ptr : nullptr, bnode_ptr ? bnode_ptr + n_bfaces + 1 : nullptr);
        H.bn.assign(bnode, bnode ? bnode + (n_bfaces ? bnode_ptr[n_bfaces] : 0) : nullptr);
        H.bt.assign(btag, btag ? btag + n_bfaces : nullptr);
        if (node_canon) H.canon.assign(node_canon, node_canon + n_nodes);
        else H.canon.clear();
    }
    c->n_params = 0;
    c->pdir_prim.clear();
    c->pdir_xyz.clear();
    if (c->prm.precision == 1) ensure_fp32_front(c);
    API_END(c)
}

cgks_status cgks_cell_order(const cgks_ctx *c, int32_t *perm)
{
    if (!c || !perm) return CGKS_E_ARG;
    if (!c->has_mesh) return CGKS_E_STATE;
    for (int64_t i = 0; i < c->N; ++i) perm[i] = (int32_t)c->caller_cell(i);
    return CGKS_OK;
}

cgks_status cgks_set_bc(cgks_ctx *c, int32_t tag, int32_t kind, const double *prim)
{
    API_BEGIN(c)
    if (c->adj) c->adj->ready = false;  // the linearisation no longer matches
    if (tag < 1 || tag > 63) throw Error{CGKS_E_ARG, "tag must be in 1..63"};
    if (kind != CGKS_BC_SLIP && kind != CGKS_BC_NOSLIP_ADIABATIC && kind != CGKS_BC_FARFIELD)
        throw Error{CGKS_E_ARG, "unknown boundary kind"};
    if (kind == CGKS_BC_FARFIELD && (!prim || !(prim[0] > 0.0) || !(prim[4] > 0.0)))
        throw Error{CGKS_E_ARG, "far field needs rho > 0 and p > 0"};
    c->bc_host.kind[tag] = kind;
    c->tags_set |= uint64_t(1) << tag;
    for (int k = 0; k < 5; ++k) c->bc_host.prim[tag][k] = prim ? prim[k] : 0.0;
    CGKS_HIP(hipMemcpyAsync(c->bc.p, &c->bc_host, sizeof(BcTable), hipMemcpyHostToDevice, c->stream));
    CGKS_HIP(hipStreamSynchronize(c->stream));
    API_END(c)
}

cgks_status cgks_mesh_info(const cgks_ctx *c, int64_t *out)
{
    if (!c || !out) return CGKS_E_ARG;
    for (int i = 0; i < 16; ++i) out[i] = 0;
    out[0] = c->N;
    out[1] = c->F;
    out[2] = c->Fi;
    out[3] = c->Fb;
    out[4] = c->NGP;
    out[5] = (int64_t)c->lev.size();
    out[6] = c->N;
    for (size_t l = 1; l < c->lev.size() && l < 8; ++l) out[6 + l] = c->lev[l]->n;
    return CGKS_OK;
}

cgks_status cgks_geometry(cgks_ctx *c, double *vol, double *cen, double *mom2)
{
    API_BEGIN(c)
    need_mesh(c);
    const size_t N = c->N;
    const double *src[3] = {c->vol.p, c->cen.p, c->mom2.p};
    double *dst[3] = {vol, cen, mom2};
    const int nc[3] = {1, 3, 6};
    for (int k = 0; k < 3; ++k) {
        if (!dst[k]) continue;
        if (io_moved(c)) cells_scatter(c, src[k], dst[k], nc[k]);
        else CGKS_HIP(hipMemcpyAsync(dst[k], src[k], nc[k] * N * 8, hipMemcpyDeviceToDevice, c->stream));
    }
    API_END(c)
}

cgks_status cgks_local_dt(cgks_ctx *c, const double *W, double *dt)
{
    API_BEGIN(c)
    need_mesh(c);
    if (!W || !dt) throw Error{CGKS_E_ARG, "null pointer"};
    double *dto = cells_buf(c, dt, 1, 6);
    launch_local_dt(c, cells_in(c, W, 5, 0), dto);
    cells_out(c, dt, 1, 6);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_reconstruct(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *coef)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !coef) throw Error{CGKS_E_ARG, "null pointer"};
    double *co = cells_buf(c, coef, 50, 6);
    launch_recon(c, cells_in(c, W, 5, 0), cells_in(c, G, 15, 1), cells_in(c, alpha, 1, 2), co, false);
    cells_out(c, coef, 50, 6);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_residual(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *R, double *G_new,
                          double *alpha_new)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !R || (G_new == nullptr) != (alpha_new == nullptr))
        throw Error{CGKS_E_ARG, "W, G, R required; G_new and alpha_new both or neither"};
    const bool fp32 = c->prm.precision == 1;
    launch_local_dt_recon(c, cells_in(c, W, 5, 0), cells_in(c, G, 15, 1), cells_in(c, alpha, 1, 2), c->dtc.p,
                          c->coef.p, nullptr, fp32 ? c->coeff.p : nullptr);
    const int mode = G_new ? MODE_RES : MODE_RESONLY;
    launch_face(c, mode, c->coef.p, c->dtc.p, -1.0, fp32);
    launch_gather_res(c, cells_buf(c, R, 5, 3), cells_buf(c, G_new, 15, 4), cells_buf(c, alpha_new, 1, 5), mode);
    cells_out(c, R, 5, 3);
    cells_out(c, G_new, 15, 4);
    cells_out(c, alpha_new, 1, 5);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_residual_noalloc(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *R,
                                  double *G_new, double *alpha_new)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !R || (G_new == nullptr) != (alpha_new == nullptr))
        throw Error{CGKS_E_ARG, "W, G, R required; G_new and alpha_new both or neither"};
    const int mode = G_new ? MODE_RES : MODE_RESONLY;
    const bool moved = io_moved(c);
    const int64_t N = c->N, F = c->F, Fb = c->F - c->Fi;
    // carve the work array: every piece 256-byte aligned
    auto up = [](int64_t n) { return (n + 31) / 32 * 32; };
    const int64_t n_dt = up(N), n_coef = up(50 * N), n_bgq = up(5 * (Fb > 0 ? Fb : 1)),
                  n_rec = up((mode == MODE_RES ? 21 : 5) * F), n_io = moved ? up(21 * N) : 0;
    const int64_t need = n_dt + n_coef + n_bgq + n_rec + 2 * n_io;
    if (need > (int64_t)SCRATCH_DOUBLES)
        throw Error{CGKS_E_ARG, "mesh too large for cgks_residual_noalloc: it needs " + std::to_string(need) +
                                    " doubles of work memory, the fixed array holds " +
                                    std::to_string(SCRATCH_DOUBLES)};
    if (c->device_now() != c->device) throw Error{CGKS_E_DEVICE, "the context's device is not the current device"};
    double *p = c->scratch;
    double *dtc = p, *coef = p + n_dt, *bgq = coef + n_coef, *rec = bgq + n_bgq, *in = rec + n_rec, *out = in + n_io;
    const double *w = W, *g = G, *a = alpha;
    double *r = R, *gn = G_new, *an = alpha_new;
    if (moved) {
        // reordered inputs and outputs: W, G, alpha and R, G_new, alpha_new (5 + 15 + 1 components)
        auto gather = [&](const double *src, double *dst, int nc) {
            hipLaunchKernelGGL(k_cells_in, dim3(blocks_for(N, 256), nc), dim3(256), 0, c->stream, N, c->perm.p, src,
                               dst);
        };
        gather(W, in, 5);
        gather(G, in + 5 * N, 15);
        w = in;
        g = in + 5 * N;
        if (alpha) {
            gather(alpha, in + 20 * N, 1);
            a = in + 20 * N;
        }
        r = out;
        gn = G_new ? out + 5 * N : nullptr;
        an = alpha_new ? out + 20 * N : nullptr;
    }
    // FP32 flux: FP32 coefficients in the same piece of the work array (50 N floats)
    const bool fp32 = c->prm.precision == 1;
    float *coef32 = fp32 ? reinterpret_cast<float *>(coef) : nullptr;
    launch_local_dt_recon(c, w, g, a, dtc, coef, bgq, coef32);
    launch_face(c, mode, coef, dtc, -1.0, fp32, rec, coef32);
    launch_gather_res(c, r, gn, an, mode, rec);
    if (moved) {
        cells_scatter(c, (const double *)out, R, 5);
        if (G_new) {
            cells_scatter(c, (const double *)(out + 5 * N), G_new, 15);
            cells_scatter(c, (const double *)(out + 20 * N), alpha_new, 1);
        }
    }
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_wall_force(cgks_ctx *c, const double *W, const double *G, const double *alpha, int32_t tag, double *F)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !F) throw Error{CGKS_E_ARG, "W, G and F required"};
    if (tag < 1 || tag > 63) throw Error{CGKS_E_ARG, "tag must be in 1..63"};
    launch_local_dt_recon(c, cells_in(c, W, 5, 0), cells_in(c, G, 15, 1), cells_in(c, alpha, 1, 2), c->dtc.p,
                          c->coef.p);
    launch_face(c, MODE_RESONLY, c->coef.p, c->dtc.p, -1.0, false);
    launch_wall_force(c, tag, F);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_linearize(cgks_ctx *c, const double *W, const double *G, const double *alpha)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G) throw Error{CGKS_E_ARG, "W and G required"};
    adj_linearize(c, cells_in(c, W, 5, 0), cells_in(c, G, 15, 1), cells_in(c, alpha, 1, 2));
    API_END(c)
}

cgks_status cgks_vjp_residual(cgks_ctx *c, const double *barR, const double *barGnew, const double *barAnew,
                              double *barW, double *barG, double *barAlpha)
{
    API_BEGIN(c)
    need_bc(c);
    if (!barR || !barW || !barG) throw Error{CGKS_E_ARG, "barR, barW and barG required"};
    adj_vjp_residual(c, cells_in(c, barR, 5, 0), cells_in(c, barGnew, 15, 1), cells_in(c, barAnew, 1, 2),
                     cells_buf(c, barW, 5, 3), cells_buf(c, barG, 15, 4), cells_buf(c, barAlpha, 1, 5), false);
    cells_out(c, barW, 5, 3);
    cells_out(c, barG, 15, 4);
    cells_out(c, barAlpha, 1, 5);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_jvp_residual(cgks_ctx *c, const double *W, const double *G, const double *alpha, const double *vW,
                              const double *vG, const double *vA, double *dR, double *dG, double *dA)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !vW || !vG || !dR) throw Error{CGKS_E_ARG, "W, G, vW, vG and dR required"};
    const double *w = cells_in(c, W, 5, 0), *g = cells_in(c, G, 15, 1), *a = cells_in(c, alpha, 1, 2);
    const double *tw = cells_in(c, vW, 5, 3), *tg = cells_in(c, vG, 15, 4), *ta = cells_in(c, vA, 1, 5);
    DBuf<double> oR, oG, oA;
    double *r = dR, *gn = dG, *an = dA;
    if (io_moved(c)) {
        oR.alloc(5 * c->N);
        r = oR.p;
        if (dG) {
            oG.alloc(15 * c->N);
            gn = oG.p;
        }
        if (dA) {
            oA.alloc(c->N);
            an = oA.p;
        }
    }
    jvp_residual(c, w, g, a, tw, tg, ta, r, gn, an);
    if (io_moved(c)) {
        cells_scatter(c, (const double *)r, dR, 5);
        if (dG) cells_scatter(c, (const double *)gn, dG, 15);
        if (dA) cells_scatter(c, (const double *)an, dA, 1);
        CGKS_HIP(hipStreamSynchronize(c->stream));
    }
    check_bad(c);
    API_END(c)
}

cgks_status cgks_vjp_wall_force(cgks_ctx *c, int32_t tag, const double *e, double *barW, double *barG,
                                double *barAlpha)
{
    API_BEGIN(c)
    need_bc(c);
    if (!e || !barW || !barG) throw Error{CGKS_E_ARG, "e, barW and barG required"};
    if (tag < 1 || tag > 63) throw Error{CGKS_E_ARG, "tag must be in 1..63"};
    adj_vjp_wall(c, tag, e, cells_buf(c, barW, 5, 3), cells_buf(c, barG, 15, 4), cells_buf(c, barAlpha, 1, 5), false);
    cells_out(c, barW, 5, 3);
    cells_out(c, barG, 15, 4);
    cells_out(c, barAlpha, 1, 5);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_vjp_kfvs(cgks_ctx *c, int32_t level, const double *Wc, const double *barRc, double *barWc)
{
    API_BEGIN(c)
    need_bc(c);
    if (!Wc || !barRc || !barWc) throw Error{CGKS_E_ARG, "null pointer"};
    adj_vjp_kfvs(c, level, Wc, barRc, barWc, false);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_set_param_directions(cgks_ctx *c, int32_t n_params, const double *dprim, const double *dxyz,
                                      double step)
{
    API_BEGIN(c)
    need_mesh(c);
    if (n_params < 0 || n_params > 8) throw Error{CGKS_E_ARG, "n_params must be in 0..8"};
    if (n_params > 0 && !(step > 0.0)) throw Error{CGKS_E_ARG, "step must be positive"};
    c->n_params = n_params;
    c->param_step = step;
    c->pdir_prim.assign((size_t)n_params * 64 * 5, 0.0);
    if (dprim) std::copy(dprim, dprim + (size_t)n_params * 64 * 5, c->pdir_prim.begin());
    c->pdir_xyz.clear();
    if (dxyz) c->pdir_xyz.assign(dxyz, dxyz + (size_t)n_params * 3 * c->hmesh.n_nodes);
    API_END(c)
}

cgks_status cgks_adjoint_solve(cgks_ctx *c, int32_t tag, const double *e, int32_t max_iter, double tol,
                               double *lamW, double *lamG, double *lamA, double *cR, double *cG, double *cA,
                               double *hist, int32_t *n_done, double *dJ_dparams)
{
    API_BEGIN(c)
    need_bc(c);
    if (!e || !n_done || max_iter < 1) throw Error{CGKS_E_ARG, "e, n_done and max_iter >= 1 required"};
    if (tag < 1 || tag > 63) throw Error{CGKS_E_ARG, "tag must be in 1..63"};
    *n_done = adj_solve(c, tag, e, max_iter, tol, cells_buf(c, lamW, 5, 0), cells_buf(c, lamG, 15, 1),
                        cells_buf(c, lamA, 1, 2), cells_buf(c, cR, 5, 3), cells_buf(c, cG, 15, 4), cells_buf(c, cA, 1, 5),
                        hist);
    cells_out(c, lamW, 5, 0);
    cells_out(c, lamG, 15, 1);
    cells_out(c, lamA, 1, 2);
    cells_out(c, cR, 5, 3);
    cells_out(c, cG, 15, 4);
    cells_out(c, cA, 1, 5);
    if (dJ_dparams && c->n_params > 0) adj_param_derivatives(c, tag, e, dJ_dparams);
    API_END(c)
}

cgks_status cgks_step(cgks_ctx *c, double *W, double *G, double *alpha, double dt_global, double *resnorm)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !alpha) throw Error{CGKS_E_ARG, "null pointer"};
    double *const Wu = W, *const Gu = G, *const Au = alpha;
    W = cells_in(c, Wu, 5, 0);
    G = cells_in(c, Gu, 15, 1);
    alpha = cells_in(c, Au, 1, 2);
    if (dt_global <= 0.0) {
        launch_local_dt_recon(c, W, G, alpha, c->dtc.p, c->coef.p);
        launch_face(c, MODE_RES, c->coef.p, c->dtc.p, -1.0, false);
        const int nb = gather_blocks(c->N);
        c->partial.ensure(nb);
        launch_gather_fe(c, W, G, alpha, c->dtc.p, c->Rw.p, c->partial.p);
        if (resnorm) finish_norm(c, c->partial.p, nb, c->N, resnorm);
    } else {
        launch_recon(c, W, G, alpha, c->coef.p);
        launch_face(c, MODE_S1, c->coef.p, nullptr, dt_global, false);
        launch_gather_s2o4(c, 1, dt_global, W, G, alpha);
        launch_recon(c, c->Ws.p, c->Gs.p, c->aw.p, c->coef.p);
        launch_face(c, MODE_S2, c->coef.p, nullptr, dt_global, false);
        launch_gather_s2o4(c, 2, dt_global, W, G, alpha);
    }
    cells_out(c, Wu, 5, 0);
    cells_out(c, Gu, 15, 1);
    cells_out(c, Au, 1, 2);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_residual_norm(cgks_ctx *c, const double *R, double *out)
{
    API_BEGIN(c)
    need_mesh(c);
    if (!R || !out) throw Error{CGKS_E_ARG, "null pointer"};
    launch_norm(c, cells_in(c, R, 5, 3), c->vol.p, c->N, out);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_check(cgks_ctx *c)
{
    API_BEGIN(c)
    need_mesh(c);
    check_bad(c);
    API_END(c)
}

cgks_status cgks_agglomerate_graph(cgks_ctx *c, int64_t n, const double *V, const double *P, int64_t m,
                                   const int32_t *pa, const int32_t *pb, const double *S, const double *M,
                                   const double *A, int32_t passes, int32_t *f2c, double *Vc, double *Pc,
                                   int64_t *n_coarse, int64_t *m_coarse, int64_t *stats)
{
    API_BEGIN(c)
    if (n <= 0 || m < 0 || n > INT32_MAX / 2 || m > INT32_MAX / 2 || passes < 0 || passes > 16)
        throw Error{CGKS_E_ARG, "graph sizes or pass count out of range"};
    if (!V || !P || !f2c || !Vc || !Pc || !n_coarse || !m_coarse || (m > 0 && (!pa || !pb || !S || !M || !A)))
        throw Error{CGKS_E_ARG, "null pointer"};
    agglomerate_graph(c, n, V, P, m, pa, pb, S, M, A, passes, f2c, Vc, Pc, n_coarse, m_coarse, stats, nullptr, nullptr,
                      nullptr, nullptr, nullptr);
    API_END(c)
}

cgks_status cgks_agglomerate(cgks_ctx *c)
{
    API_BEGIN(c)
    if (c->adj) c->adj->ready = false;  // the linearisation no longer matches
    need_mesh(c);
    build_hierarchy(c);
    API_END(c)
}

static Level *level_at(cgks_ctx *c, int32_t level)
{
    if (level < 1 || level >= (int32_t)c->lev.size()) throw Error{CGKS_E_STATE, "level not built (cgks_agglomerate)"};
    return c->lev[level];
}

cgks_status cgks_level_map(cgks_ctx *c, int32_t level, int32_t *f2c)
{
    API_BEGIN(c)
    need_mesh(c);
    Level *L = level_at(c, level);
    if (!f2c) throw Error{CGKS_E_ARG, "null pointer"};
    if (level == 1 && io_moved(c)) cells_scatter(c, L->f2c.p, f2c, 1);
    else CGKS_HIP(hipMemcpyAsync(f2c, L->f2c.p, 4 * L->nfine, hipMemcpyDeviceToDevice, c->stream));
    API_END(c)
}

cgks_status cgks_kfvs_residual(cgks_ctx *c, int32_t level, const double *W, double *R)
{
    API_BEGIN(c)
    need_bc(c);
    level_at(c, level);
    if (!W || !R) throw Error{CGKS_E_ARG, "null pointer"};
    if (c->prm.precision == 1) kfvs_residual_fp32(c, level, W, R);
    else kfvs_residual(c, level, W, R);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_coarse_implicit(cgks_ctx *c, int32_t level, const double *W, const double *rhs, double *dU)
{
    API_BEGIN(c)
    need_bc(c);
    level_at(c, level);
    if (!W || !rhs || !dU) throw Error{CGKS_E_ARG, "null pointer"};
    if (!(c->prm.cfl_implicit > 0.0)) throw Error{CGKS_E_ARG, "cfl_implicit must be positive"};
    if (c->prm.precision == 1) coarse_implicit_fp32(c, level, W, rhs, dU);
    else coarse_implicit(c, level, W, rhs, dU);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_restrict(cgks_ctx *c, int32_t level, const double *Wf, const double *Rf, double *Wc, double *Rc)
{
    API_BEGIN(c)
    need_mesh(c);
    level_at(c, level);
    if ((Wf == nullptr) != (Wc == nullptr) || (Rf == nullptr) != (Rc == nullptr))
        throw Error{CGKS_E_ARG, "each of (Wf, Wc) and (Rf, Rc) must be both set or both null"};
    if (level == 1) {
        Wf = cells_in(c, Wf, 5, 0);
        Rf = cells_in(c, Rf, 5, 3);
    }
    restrict_level(c, level, Wf, Rf, Wc, Rc);
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_prolong(cgks_ctx *c, int32_t level, const double *dWc, double *Wf)
{
    API_BEGIN(c)
    need_mesh(c);
    level_at(c, level);
    if (!dWc || !Wf) throw Error{CGKS_E_ARG, "null pointer"};
    if (level == 1) {
        double *w = cells_in(c, Wf, 5, 0);
        prolong_level(c, level, dWc, w);
        cells_out(c, Wf, 5, 0);
    } else {
        prolong_level(c, level, dWc, Wf);
    }
    CGKS_HIP(hipGetLastError());
    API_END(c)
}

cgks_status cgks_vcycle(cgks_ctx *c, double *W, double *G, double *alpha, int32_t max_cycles, double tol_drop,
                        double *hist, int32_t *n_done)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !alpha || max_cycles < 0) throw Error{CGKS_E_ARG, "bad arguments"};
    // the cycles run on the internal order; the state goes back to the caller's order on every
    // exit, a stop, an error or a state error included
    double *w = cells_in(c, W, 5, 0), *g = cells_in(c, G, 15, 1), *a = cells_in(c, alpha, 1, 2);
    cgks_status st;
    try {
        st = vcycle_impl(c, w, g, a, max_cycles, tol_drop, hist, n_done);
    } catch (...) {
        cells_out(c, W, 5, 0);
        cells_out(c, G, 15, 1);
        cells_out(c, alpha, 1, 2);
        throw;
    }
    cells_out(c, W, 5, 0);
    cells_out(c, G, 15, 1);
    cells_out(c, alpha, 1, 2);
    if (st != CGKS_OK) return st;
    API_END(c)
}

// ---------------------------------------------------------------- host-pointer twins
cgks_status cgks_residual_host(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *R,
                               double *G_new, double *alpha_new)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !R || (G_new == nullptr) != (alpha_new == nullptr))
        throw Error{CGKS_E_ARG, "W, G, R required; G_new and alpha_new both or neither"};
    const int64_t N = c->N;
    DBuf<double> w, g, a, r, gn, an;
    w.upload(W, 5 * N, c->stream);
    g.upload(G, 15 * N, c->stream);
    if (alpha) a.upload(alpha, N, c->stream);
    r.alloc(5 * N);
    if (G_new) {
        gn.alloc(15 * N);
        an.alloc(N);
    }
    const cgks_status st = cgks_residual(c, w.p, g.p, alpha ? a.p : nullptr, r.p, gn.p, an.p);
    if (st != CGKS_OK) return st;
    CGKS_HIP(hipMemcpyAsync(R, r.p, 5 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (G_new) {
        CGKS_HIP(hipMemcpyAsync(G_new, gn.p, 15 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        CGKS_HIP(hipMemcpyAsync(alpha_new, an.p, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    }
    CGKS_HIP(hipStreamSynchronize(c->stream));
    check_bad(c);
    API_END(c)
}

cgks_status cgks_vcycle_host(cgks_ctx *c, double *W, double *G, double *alpha, int32_t max_cycles, double tol_drop,
                             double *hist, int32_t *n_done)
{
    API_BEGIN(c)
    need_bc(c);
    if (!W || !G || !alpha || max_cycles < 0) throw Error{CGKS_E_ARG, "bad arguments"};
    const int64_t N = c->N;
    DBuf<double> w, g, a;
    w.upload(W, 5 * N, c->stream);
    g.upload(G, 15 * N, c->stream);
    a.upload(alpha, N, c->stream);
    const cgks_status st = cgks_vcycle(c, w.p, g.p, a.p, max_cycles, tol_drop, hist, n_done);
    if (st != CGKS_OK && st != CGKS_E_NOCONV && st != CGKS_E_PHYS && st != CGKS_E_NONFINITE) return st;
    const std::string msg = c->err;
    CGKS_HIP(hipMemcpyAsync(W, w.p, 5 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CGKS_HIP(hipMemcpyAsync(G, g.p, 15 * N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CGKS_HIP(hipMemcpyAsync(alpha, a.p, N * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    CGKS_HIP(hipStreamSynchronize(c->stream));
    if (st != CGKS_OK) {
        c->err = msg;
        return st;
    }
    API_END(c)
}

cgks_status cgks_timing(cgks_ctx *c, int32_t enable, double *face_ms, int64_t *face_launches)
{
    API_BEGIN(c)
    if (enable) {
        c->timing = true;
        c->ev_used = 0;
    } else {
        CGKS_HIP(hipStreamSynchronize(c->stream));
        double ms = 0.0;
        for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
            float t = 0.f;
            CGKS_HIP(hipEventElapsedTime(&t, c->ev_pool[k], c->ev_pool[k + 1]));
            ms += t;
        }
        if (face_ms) *face_ms = ms;
        if (face_launches) *face_launches = (int64_t)(c->ev_used / 2);
        c->timing = false;
        c->ev_used = 0;
    }
    API_END(c)
}

}  // extern "C"

// Library internals shared by the translation units of libcgks.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/cgks.h"

namespace cgks {

struct Error {
    cgks_status code;
    std::string msg;
};

#define CGKS_HIP(expr)                                                                                   \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess)                                                                            \
            throw ::cgks::Error{CGKS_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)};      \
    } while (0)

template <class T> struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    void alloc(size_t count)
    {
        release();
        if (!count) return;
        const hipError_t e = hipMalloc(&p, sizeof(T) * count);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();  // a refused allocation must not surface again at a later check
            throw ::cgks::Error{CGKS_E_DEVICE, "hipMalloc of " + std::to_string(sizeof(T) * count) +
                                                   " bytes: " + hipGetErrorString(e)};
        }
        n = count;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void ensure(size_t count)
    {
        if (n < count) alloc(count);
    }
    void upload(const T *h, size_t count, hipStream_t s)
    {
        ensure(count);
        if (count) CGKS_HIP(hipMemcpyAsync(p, h, sizeof(T) * count, hipMemcpyHostToDevice, s));
    }
    void upload(const std::vector<T> &v, hipStream_t s) { upload(v.data(), v.size(), s); }
    std::vector<T> download(size_t count, hipStream_t s) const
    {
        std::vector<T> v(count);
        if (count) {
            CGKS_HIP(hipMemcpyAsync(v.data(), p, sizeof(T) * count, hipMemcpyDeviceToHost, s));
            CGKS_HIP(hipStreamSynchronize(s));
        }
        return v;
    }
    ~DBuf() { release(); }
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
};

// Boundary table kept in device memory, indexed by tag.
struct BcTable {
    int32_t kind[64];
    double prim[64][5];
};

// One coarse level (l >= 1) of the hierarchy.
struct Level {
    int64_t n = 0, m = 0, nb = 0, nfine = 0;
    int64_t nnz = 0;                 // entries of the cell -> face list
    DBuf<int32_t> f2c;               // [nfine] from level l-1
    DBuf<int32_t> c2f_ptr, c2f_idx;  // CSR coarse -> fine, fine ids ascending
    DBuf<double> V;                  // [n]
    DBuf<double> P;                  // [3n] interleaved first moments
    DBuf<int32_t> pa, pb;            // [m] coarse interior pairs
    DBuf<double> S;                  // [m] summed fine areas
    DBuf<double> A;                  // [3][m] summed area vectors (SoA)
    DBuf<double> AS;                 // [m][4] area vector and summed area, interleaved (row kernels)
    DBuf<int32_t> bown, btag;        // [nb] coarse owner, tag of the fine boundary faces
    DBuf<double> bA;                 // [3][nb]
    DBuf<int32_t> cf_ptr, cf_item;   // CSR cell -> (pair j: 2j + side) / (boundary k: -(k+1))
    // work buffers (FP64)
    DBuf<double> W0, W, D, R, F, Rs, dt, fflux;
    // FP32 work buffers (mixed precision)
    DBuf<float> W0f, Wf, Df, Rf, Ff, Rsf, dtf, ffluxf;
    // implicit smoother: lambda S / 2 per cell-face entry, diagonal, two relaxation iterates
    DBuf<double> lamS, dg, dUa, dUb;
    DBuf<float> lamSf, dgf, dUaf, dUbf;
};

// Linearisation of the fine operator at one state, kept for repeated
// vector-Jacobian products (the discrete adjoint).  Sizes: NS = 4F Gauss-point
// slots, N cells, F faces.
struct AdjTape {
    bool ready = false;
    DBuf<double> W, G, al;     // linearisation point (5N, 15N, N)
    DBuf<double> dt, ddt;      // local step (N) and its derivative w.r.t. the own state (5N)
    DBuf<uint8_t> dtL;         // [F] 1: the face step is the left cell's
    DBuf<double> coef;         // cell-major polynomial coefficients (50N)
    DBuf<double> rec;          // face records of the full mode (21F)
    DBuf<double> Anew, Sgv;    // CF product per cell (N), sum w S W n / |Omega| (15N)
    DBuf<double> agp;          // CF factor per Gauss-point slot (NS)
    bool fp32 = false;         // Jacobians stored in FP32 (params.adjoint_tape = 1)
    DBuf<double> Jf;           // Gauss-point Jacobians, 11*41 per compact Gauss point, 64-column tiles
    DBuf<double> Jr;           // reconstruction Jacobians, 10*30 per (cell, component) column (jr_at)
    DBuf<float> Jf32, Jr32;    // the same in FP32
    DBuf<int8_t> rev;          // [6][N] slot of the same face in the neighbour's list
    // cotangent work buffers
    DBuf<double> brec, bface, bcoef, bdt, bown, bslot, bat;
    // coarse levels at the linearisation point (restricted states and steps), level l at index l
    std::vector<DBuf<double> *> cW, cdt;
    // adjoint iteration work
    DBuf<double> lam, lam1, tmp, bR, jv, cR, cG, cA, part;
    std::vector<DBuf<double> *> cD, cRs, cX;
    ~AdjTape()
    {
        for (auto *b : cW) delete b;
        for (auto *b : cdt) delete b;
        for (auto *b : cD) delete b;
        for (auto *b : cRs) delete b;
        for (auto *b : cX) delete b;
    }
};

}  // namespace cgks

struct cgks_ctx {
    cgks_params prm{};
    hipStream_t stream = nullptr;
    std::string err;
    int device = 0;
    int gpu_cus = 256;

    // fine mesh sizes
    int64_t N = 0, F = 0, Fi = 0, Fb = 0, NGP = 0;
    bool has_mesh = false;
    uint64_t tags_used = 0;  // bit t: the mesh has boundary faces with tag t
    uint64_t tags_set = 0;   // bit t: a boundary condition was given for tag t

    // Internal cell order: cells are stored in a locality order (params.cell_order >= 1), the
    // caller's order otherwise.  perm[i] = caller id of internal cell i (identity when not
    // permuted); cell arrays crossing the ABI are gathered from / scattered to caller order unless
    // params.cell_order == 2 (arrays exchanged in the internal order).
    bool permuted = false;
    std::vector<int32_t> perm_h;
    cgks::DBuf<int32_t> perm;
    cgks::DBuf<double> io[8];  // staging buffers of the ABI gathers and scatters
    int64_t caller_cell(int64_t i) const
    {
        return permuted && i >= 0 && i < (int64_t)perm_h.size() ? perm_h[i] : i;
    }

    // Host copy of the mesh as built (cells in the internal order), kept for the parameter
    // sensitivities of the adjoint, which rebuild the geometry at displaced nodes.
    struct HostMesh {
        int64_t n_nodes = 0, n_bf = 0;
        std::vector<double> xyz;
        std::vector<uint8_t> ct;
        std::vector<int64_t> cp, cn, bp, bn, canon;
        std::vector<int32_t> bt;
    } hmesh;
    // parameter directions of the adjoint (cgks_set_param_directions): per parameter the derivative
    // of every tag's far-field primitives and of every node's coordinates
    int32_t n_params = 0;
    double param_step = 1e-6;
    std::vector<double> pdir_prim;  // [n_params][64][5]
    std::vector<double> pdir_xyz;   // [n_params][3 n_nodes]; empty when no parameter moves the nodes

    // fine geometry (internal cell order)
    cgks::DBuf<double> vol, cen, mom2;  // [N], [3][N], [6][N]
    cgks::DBuf<int32_t> fl, fr, ftag;   // [F]
    cgks::DBuf<int32_t> fngp;           // [F] 3 or 4
    cgks::DBuf<int32_t> gpoff;          // [F] first Gauss point of the face in a compact numbering (NGP)
    cgks::DBuf<int32_t> lmap;           // [NL] face-kernel lane -> 4 face + Gauss point, -1 idle
    int64_t NL = 0;                     // lanes of the face kernel (multiple of 256)
    cgks::DBuf<int4> lidx;              // [NL] {4 f + k, L, R, 8 tag + ngp}, f = -1 idle
    cgks::DBuf<double> lgeo;            // [10][NL] dx_L (3), dx_R (3), n (3), w S, lane-major
    cgks::DBuf<double> gpx, gpw, gpn;   // [4*3][F], [4][F] (w_k S), [4*3][F]
    cgks::DBuf<double> fshift, favec, farea, fmom;  // [3][F], [3][F], [F], [3][F]
    cgks::DBuf<int32_t> cf_ptr, cf_face;  // CSR cell -> 2*face + (cell is R)
    // reconstruction structures
    cgks::DBuf<int32_t> slot_nb;   // [6][N] neighbour cell, or -(face+1) for a boundary face, or INT32_MIN unused
    cgks::DBuf<double> slot_av;    // [6*3][N] outward area vector / |Omega|
    cgks::DBuf<int64_t> op_off;    // [N] first entry of the cell's operator (stride 64), -1: Green-Gauss only
    cgks::DBuf<uint8_t> n_int;     // [N] interior neighbours
    cgks::DBuf<double> op;         // per interior neighbour 39 entries (9 x 4 KKT columns, 3 LS), 64-cell interleaved
    cgks::DBuf<int64_t> op_gbase;  // [ceil(N/64)] first entry of each 64-cell group
    cgks::DBuf<int32_t> op_gnb;    // [ceil(N/64)] largest interior-neighbour count of the group's p^2 cells
    cgks::DBuf<int32_t> inb;       // [6][N] interior neighbours in slot order, -1 past the last
    cgks::DBuf<int32_t> op_gmax;   // [ceil(N/64)] largest interior-neighbour count of the group
    cgks::DBuf<double> iav;        // [6*3][N] area vector / |Omega| of the interior faces, in that order
    cgks::DBuf<uint8_t> nface;     // [N] faces of the cell
    cgks::DBuf<double> bgq;        // [5][Fb] ghost states of the boundary faces (reconstruction work)
    // boundary conditions
    cgks::BcTable bc_host{};
    cgks::DBuf<cgks::BcTable> bc;
    // work buffers
    cgks::DBuf<double> coef, dtc, fout, Rw, Gw, aw, Ws, Gs, L1, Lt1, Gc1, partial, scal;
    // mixed precision: FP32 copies of op and lgeo, FP32 cell-major coefficients (ensure_fp32_front)
    cgks::DBuf<float> opf, lgeof, coeff;
    cgks::DBuf<int32_t> bad;
    // multigrid hierarchy; lev[0] is a placeholder for the fine level
    std::vector<cgks::Level *> lev;
    // optional face-kernel timing (events recorded around each launch)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    // discrete-adjoint linearisation (allocated by cgks_linearize)
    cgks::AdjTape *adj = nullptr;
    // host pinned scalar for per-cycle reads
    double *pinned = nullptr;
    cgks::DBuf<double> hist_dev;                // per-cycle residual norms of a batch of V-cycles
    cgks::DBuf<double> snapW, snapG, snapA;     // state at the start of the batch
    int32_t *pinned_i = nullptr;
    // device address of the no-allocation entry point's work array on this context's device
    double *scratch = nullptr;
    int device_now() const
    {
        int d = -1;
        return hipGetDevice(&d) == hipSuccess ? d : -1;
    }

    ~cgks_ctx();
};

namespace cgks {

// launch helpers (defined in the translation units that own the kernels)
void mesh_build(cgks_ctx *c, int64_t n_nodes, const double *xyz, int64_t n_cells, const uint8_t *ctype,
                const int64_t *cptr, const int64_t *cnode, int64_t n_bf, const int64_t *bptr, const int64_t *bnode,
                const int32_t *btag, const int64_t *canon);
void launch_local_dt(cgks_ctx *c, const double *W, double *dt);
// cell-major: coef[50 i + 10 c + k], else coef[(10 c + k) N + i]; ghosts_ready: the boundary
// ghost states at W are already in bgq
// bgq: where the boundary ghost states go (nullptr: the context's buffer)
// coef32: write FP32 cell-major coefficients there instead, from the FP32 operator copy (the
// mixed-precision flux phase; coef is then unused)
void launch_recon(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *coef,
                  bool cell_major = true, bool ghosts_ready = false, double *bgq = nullptr, float *coef32 = nullptr);
// launch_local_dt + launch_recon (cell-major) with the ghost states formed in the local-step launch
void launch_local_dt_recon(cgks_ctx *c, const double *W, const double *G, const double *alpha, double *dt,
                           double *coef, double *bgq = nullptr, float *coef32 = nullptr);
enum FaceMode { MODE_RES = 0, MODE_RESONLY = 1, MODE_S1 = 2, MODE_S2 = 3 };
// out: face records (nullptr: the context's buffer; a launch with its own buffer is never timed)
// fp32: the per-point evaluation in FP32 from coef32 (nullptr: the context's FP32 coefficients)
void launch_face(cgks_ctx *c, int mode, const double *coef, const double *dt_cell, double dt_global, bool fp32,
                 double *out = nullptr, const float *coef32 = nullptr);
// FP32 copies of the reconstruction operator and the lane geometry, and the FP32 coefficient
// buffer, made once per mesh when the mixed precision is first selected
void ensure_fp32_front(cgks_ctx *c);
void launch_gather_res(cgks_ctx *c, double *R, double *Gn, double *an, int mode, const double *fout = nullptr);
void launch_gather_fe(cgks_ctx *c, double *W, double *G, double *alpha, const double *dt, double *Rout, double *norm_part);
void launch_gather_s2o4(cgks_ctx *c, int stage, double dt, double *W, double *G, double *alpha);
void launch_norm(cgks_ctx *c, const double *R, const double *vol, int64_t n, double *out);
void launch_wall_force(cgks_ctx *c, int32_t tag, double *out);  // after a MODE_RESONLY face launch
void finish_norm(cgks_ctx *c, const double *partials, int nblocks, int64_t n, double *out);
int norm_blocks(int64_t n);
int gather_blocks(int64_t n);  // blocks (and norm partials) of the FE gather
void launch_fill(double *p, double v, int64_t n, hipStream_t s);

// coarse levels
void agglomerate_graph(cgks_ctx *c, int64_t n, const double *V, const double *P, int64_t m, const int32_t *pa,
                       const int32_t *pb, const double *S, const double *M, const double *A, int passes, int32_t *f2c,
                       double *Vc, double *Pc, int64_t *n_coarse, int64_t *m_coarse, int64_t *stats,
                       // optional coarse-pair outputs (device, sized m): pairs, summed S, M (interleaved), A (interleaved)
                       int32_t *pa_out, int32_t *pb_out, double *S_out, double *M_out, double *A_out);
void build_hierarchy(cgks_ctx *c);
void kfvs_residual(cgks_ctx *c, int level, const double *W, double *R);
void kfvs_residual32(cgks_ctx *c, int level, const float *W, float *R);
void kfvs_residual_fp32(cgks_ctx *c, int level, const double *W, double *R);
void coarse_implicit(cgks_ctx *c, int level, const double *W, const double *rhs, double *dU);
void coarse_implicit_fp32(cgks_ctx *c, int level, const double *W, const double *rhs, double *dU);
void restrict_level(cgks_ctx *c, int level, const double *Wf, const double *Rf, double *Wc, double *Rc);
void prolong_level(cgks_ctx *c, int level, const double *dWc, double *Wf);
// norm_out: where the first smoothing sweep's residual norm goes (one double on the device)
void vcycle_once(cgks_ctx *c, double *W, double *G, double *alpha, bool fp32_flux, bool fp32_coarse,
                 double *norm_out);
struct GksCfg;
GksCfg cfg_of(const cgks_ctx *c);
void coarse_dt_level(cgks_ctx *c, int level, const double *W, double *dt);

// discrete adjoint
void adj_linearize(cgks_ctx *c, const double *W, const double *G, const double *alpha);
void adj_vjp_residual(cgks_ctx *c, const double *bR, const double *bG, const double *bA, double *oW, double *oG,
                      double *oA, bool accumulate);
void adj_vjp_wall(cgks_ctx *c, int32_t tag, const double e[3], double *oW, double *oG, double *oA, bool accumulate);
void adj_vjp_kfvs(cgks_ctx *c, int level, const double *Wc, const double *bR, double *oW, bool accumulate);
int adj_solve(cgks_ctx *c, int32_t tag, const double e[3], int max_iter, double tol, double *lamW, double *lamG,
              double *lamA, double *cR, double *cG, double *cA, double *hist);
// directional derivative of the fine operator by forward-mode dual numbers (no recorded Jacobian)
void jvp_residual(cgks_ctx *c, const double *W, const double *G, const double *alpha, const double *vW,
                  const double *vG, const double *vA, double *dR, double *dG, double *dA);
// after adj_solve: dJ/dp_k = dJ/dp_k|_U + c . dE/dp_k|_U for every parameter direction (host out[n_params])
void adj_param_derivatives(cgks_ctx *c, int32_t tag, const double e[3], double *out);

inline int blocks_for(int64_t n, int bs) { return (int)((n + bs - 1) / bs); }

}  // namespace cgks

// Internal state of a built mesh, shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/stdg.h"
#include "fem.hpp"

namespace stdg {

void set_error(const std::string& msg);

#define STDG_HIP(call)                                                        \
    do {                                                                      \
        hipError_t e_ = (call);                                               \
        if (e_ != hipSuccess) {                                               \
            ::stdg::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
            return STDG_ERR_DEVICE;                                           \
        }                                                                     \
    } while (0)

struct Face {
    int64_t left, right;     // internal element ids, right = -1 on a boundary
    int32_t lf, rf;          // local face index in each element
    V3 shift;                // right element's coordinates + shift = adjacent to left
};

// Device buffers owned by the handle (freed with it).
struct DeviceTables {
    double* blocks = nullptr;     // [n_classes][5][N][N]  dt^2 S^sp blocks
    float* blocks32 = nullptr;    // same, FP32
    float* aop32 = nullptr;       // FP32 blocks per lane in MFMA operand order (fused CG kernel)
    int cg_precond_ok = 0;        // every own block SPD: block-Jacobi operands in aop32
    // chunk-staged CG iteration (one workgroup per chunk of 384 consecutive
    // elements and time node; chunk_hmax = 0: not used for this mesh)
    int16_t* chunk_slot = nullptr;  // [E][4] LDS row of the neighbour across local face f, -1 none
    int32_t* chunk_halo = nullptr;  // [chunks][chunk_hmax] element of halo row h, -1 padding
    int chunk_hmax = 0;             // halo rows per chunk (multiple of 64)
    int64_t chunk_chunks = 0;
    float* elem_ops = nullptr;    // per-element FP32 blocks of the per-element PCG iteration (null: not used)
    double* elem_ops64 = nullptr; // per-element FP64 operator blocks of the FP64 apply on such meshes
    float* lane_ops = nullptr;    // class operands of the element-per-lane kernels (null: a run mixes classes)
    int runs_uniform = 0;         // every 64-element run of the element order holds one class
    int32_t* run_cls = nullptr;   // [runs] class of a one-class 64-element run, -1 for a run of several
    int32_t* mixed_elems = nullptr;   // elements of the runs of several classes
    int64_t n_mixed_elems = 0;
    int64_t n_mixed_runs = 0;
    int32_t* cls = nullptr;       // [E]
    int32_t* nbr = nullptr;       // [E][4]  -1 on a boundary face
    double* C = nullptr;          // [G][G]  time factor W T^-1 W
    float* C32 = nullptr;
    double* Cinv = nullptr;       // [G][G]  its inverse
    float* Cinv32 = nullptr;
    double* Cid = nullptr;        // [G][G]  identity (spatial operator on every time node)
    float* Cid32 = nullptr;
};

// Krylov workspaces (allocated on first solve, sized for the mesh).
struct Workspace {
    size_t n = 0;                 // vector length E*G*N
    int restart = 0;
    double* r = nullptr; double* p = nullptr; double* q = nullptr; double* z = nullptr;
    double* V = nullptr;          // GMRES basis [(m+1)][n]
    float* r32 = nullptr; float* p32 = nullptr; float* q32 = nullptr; float* x32 = nullptr;
    float* b32 = nullptr;
    float* V32 = nullptr;         // FP32 GMRES basis
    float* p32b = nullptr;        // second buffers of r, p, q (one-kernel CG iteration)
    float* r32b = nullptr;
    float* q32b = nullptr;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};   // residual checks, loop timing
    double* partial = nullptr;    // reduction partials
    double* scal = nullptr;       // device scalars (small)
    double* hscal = nullptr;      // pinned host mirror
    int64_t partial_len = 0;
};

V3 centroid(const std::array<V3, 4>& v);
int set_geometry(stdg_mesh* m, const double* nodes);        // curved elements (Sec. 2.8)
V3 neighbour_shift(const stdg_mesh* m, int64_t t, int f);   // brings the neighbour next to t
void taylor_eval(const std::vector<std::array<int, 3>>& ex, const V3& x, const V3& x0, real h, real* out);

// Spatial tables of the Picard step (Sec. 2.6), per element class c and
// local face f, row-major N x N blocks (see picard_tables.cpp).
struct PicardTables {
    std::vector<double> A, GB, QT, US, UN, BB, SV, MI;
    std::vector<double> DV;        // [C][NG][NG] inverse viscous diagonal block, column-major
    int qs = 0, qt = 0, qv = 0, nqf = 0, nqv = 0;
    std::vector<double> cJinv, cdet, cnrm, PHf, PHn, FW, PHv, dPHv, wv, tq, tw, gq;
    std::vector<double> Tm, TW, W, g0g1, g1;
};

struct PicardDevice {
    double *A = nullptr, *GB = nullptr, *QT = nullptr, *US = nullptr, *UN = nullptr, *BB = nullptr;
    double *SVT = nullptr, *MIT = nullptr, *DV = nullptr;
    double *SVt = nullptr, *MIt = nullptr;   // blocks transposed (column-major) for the register kernels
    double *At = nullptr, *GBt = nullptr, *QTt = nullptr, *USt = nullptr, *UNt = nullptr, *BBt = nullptr;
    double *cJinv = nullptr, *cdet = nullptr, *cnrm = nullptr, *PHf = nullptr, *PHn = nullptr, *FW = nullptr;
    double *PHv = nullptr, *dPHv = nullptr, *wv = nullptr, *tq = nullptr, *tw = nullptr, *gq = nullptr;
    double *Tm = nullptr, *TW = nullptr, *W = nullptr, *g0g1 = nullptr, *g1 = nullptr;
    int64_t* tet_face = nullptr;     // [E][4]
    int64_t* fl = nullptr;           // [F] left element
    int64_t* fr = nullptr;           // [F] right element (-1 boundary)
    int32_t* flf = nullptr;          // [F] left local face
    int32_t* frf = nullptr;          // [F] right local face
    double* work = nullptr;          // step workspace
    size_t work_len = 0;
    double* conv_tmp = nullptr;      // convection sums per time point [qt][3][E][N]
    size_t conv_len = 0;
};

}  // namespace stdg

struct stdg_mesh {
    stdg_config cfg;
    int p = 0, G = 0, N = 0, Nst = 0;
    int64_t E = 0;
    std::vector<int64_t> perm;        // internal -> input
    std::vector<int64_t> iperm;       // input -> internal
    std::vector<std::array<stdg::V3, 4>> vert;   // internal order, local vertex order kept
    std::vector<stdg::V3> geo;        // [E][N] isoparametric nodes (curved meshes), internal order
    std::vector<uint8_t> bent;        // [E] 1: the element's nodes are not an affine image
    bool curved = false;              // some element is bent (Picard tables are not built)
    std::vector<int32_t> nbr;         // [E][4]
    std::vector<int64_t> tet_face;    // [E][4] face id
    std::vector<stdg::Face> faces;    // interior first, then boundary
    int64_t n_interior = 0;
    std::vector<int32_t> cls;         // [E]
    int n_classes = 0;
    std::vector<double> blocks;       // [n_classes][5][N][N]
    std::vector<double> Ctime;        // [G][G]
    int64_t anchor = 0;               // internal anchor element
    int anchor_node = 0;
    stdg::DeviceTables d;
    stdg::Workspace ws;
    stdg::PicardTables pt;
    stdg::PicardDevice pd;
};

// Launch wrappers shared between the library's HIP translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/stdg.h"

struct stdg_mesh;

namespace stdg {

hipError_t launch_apply_f64(const stdg_mesh* m, const double* x, double* y, hipStream_t s);
hipError_t launch_apply_f32(const stdg_mesh* m, const float* x, float* y, hipStream_t s);
hipError_t launch_apply_f64_c(const stdg_mesh* m, const double* C, const double* x, double* y,
                              hipStream_t s);
hipError_t launch_apply_f32_c(const stdg_mesh* m, const float* C, const float* x, float* y, hipStream_t s);
constexpr int CG_UPD_BLOCKS = 1024;
bool cg_fused_supported(const stdg_mesh* m);
int upload_cg_operands(stdg_mesh* m);
int64_t cg_op_blocks(const stdg_mesh* m);
int64_t cg_partial_len(const stdg_mesh* m);   // doubles of one launch's partials
hipError_t launch_cg_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                              float* r_out, float* p_out, float* q_out, int iter, float cscale, bool precond,
                              const double* part_in, int64_t n_in, double* part_out, double* ab, hipStream_t s);
hipError_t launch_cg_prec_f32(const stdg_mesh* m, const float* x, float* y, float scale, hipStream_t s);
hipError_t launch_cg_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s);
hipError_t launch_cg_tail_f32(float* x, const float* p, int64_t n, const double* part, int64_t n_part, double* ab,
                              hipStream_t s);
bool elem_supported(const stdg_mesh* m);
int upload_elem_operands(stdg_mesh* m, const std::vector<double>& inv);
int64_t elem_iter_blocks(const stdg_mesh* m);
bool elem_apply64_supported(const stdg_mesh* m);
hipError_t elem_apply_f64(const stdg_mesh* m, const double* C, const double* x, double* y, hipStream_t s);
hipError_t elem_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s);
hipError_t elem_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                         float* r_out, float* p_out, float* q_out, const double* ab, float cscale, int precond,
                         double* part_out, hipStream_t s);
bool lane_supported(const stdg_mesh* m);
int upload_lane_operands(stdg_mesh* m, const std::vector<double>& inv);
int64_t lane_iter_blocks(const stdg_mesh* m);
hipError_t lane_iter_f32(const stdg_mesh* m, float* x, const float* r_in, const float* p_in, const float* q_in,
                         float* r_out, float* p_out, float* q_out, const double* ab, float cscale, int precond,
                         double* part_out, hipStream_t s);
hipError_t lane_apply_f32(const stdg_mesh* m, const float* x, float* y, float cscale, hipStream_t s);
hipError_t lane_prec_f32(const stdg_mesh* m, const float* x, float* y, float scale, hipStream_t s);
int64_t lane_len(const stdg_mesh* m);   // floats of a run-layout vector
hipError_t lane_pack(const stdg_mesh* m, const double* x, double scale, float* y, hipStream_t s);
hipError_t lane_unpack(const stdg_mesh* m, const float* y, const double* M, double scale, bool add, double* x,
                       hipStream_t s);
hipError_t launch_cg_check_f32(const double* part, int64_t n_part, double* scal, int slot, hipStream_t s);
hipError_t time_mix_f64(const stdg_mesh* m, const double* M, const double* x, double* y, hipStream_t s);
hipError_t time_mix_f32(const stdg_mesh* m, const float* M, const float* x, float* y, hipStream_t s);
hipError_t launch_visc_apply(const stdg_mesh* m, const double* x, double* y, hipStream_t s);
int model_predict(stdg_model* md, const stdg_mesh* m, const double* P, const double* Pm, const double* B,
                  double* x0, hipStream_t s, bool correction_only);
int device_dots(stdg_mesh* m, int k, const double* const* a, const double* const* b, int64_t n, hipStream_t s,
                double* out);
bool fast_rows_supported(const stdg_mesh* m);
hipError_t fast_convection(const stdg_mesh* m, const double* vbar, const double* vbc, double* ups, hipStream_t s);
hipError_t fast_dualgrad(const stdg_mesh* m, const double* p, double dt, double* w, hipStream_t s);
hipError_t fast_goback(const stdg_mesh* m, const double* vbar, const double* vbdry, double* out, int64_t f0,
                       int64_t f1, hipStream_t s);
hipError_t fast_average(const stdg_mesh* m, const double* vhat, double* vbar, hipStream_t s);
hipError_t fast_rhs_pressure(const stdg_mesh* m, const double* Fv, double dt, double* b, hipStream_t s);
hipError_t fast_visc_rhs(const stdg_mesh* m, const double* vprev, const double* ups, const double* lam,
                         const double* vbc, double* rhs, hipStream_t s);
hipError_t fast_blockdiag(const stdg_mesh* m, const double* x, double* y, hipStream_t s);
hipError_t launch_visc_precond(const stdg_mesh* m, const double* x, double* y, hipStream_t s);
hipError_t convert_d2f(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t convert_f2d(const float* a, double* b, int64_t n, hipStream_t s);

int build_topology(stdg_mesh* m, const double* xyz, int64_t n_vert, const int64_t* tets,
                   const std::vector<int64_t>* order);
int assign_classes(stdg_mesh* m, std::vector<int64_t>& rep);
std::vector<int64_t> class_chunk_order(const stdg_mesh* m);
void sort_faces_by_class(stdg_mesh* m);
int build_blocks(stdg_mesh* m, const std::vector<int64_t>& rep);
int upload_tables(stdg_mesh* m);
void free_tables(stdg_mesh* m);
int build_picard_tables(stdg_mesh* m, const std::vector<int64_t>& rep);
int upload_picard_tables(stdg_mesh* m);
void free_picard(stdg_mesh* m);
int viscous_solve(stdg_mesh* m, const double* b, double* x, const stdg_solve_opts& o, double* work,
                  hipStream_t s, int& iters, double& rel);

}  // namespace stdg

// C ABI entry points: mesh handle life cycle, operator application, errors.
#include <cstring>
#include <exception>
#include <new>
#include <string>

#include <algorithm>

#include "internal.hpp"
#include "kernels.hpp"

namespace stdg {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

void free_workspace(stdg_mesh* m);

int upload_tables(stdg_mesh* m) {
    // device layout: each N x N block transposed (BT[c][k][m][r] = B[c][k][r][m])
    const int N = m->N;
    const size_t nb = (size_t)m->n_classes * 5 * N * N;
    std::vector<double> bt(nb);
    std::vector<float> b32(nb);
    for (size_t blk = 0; blk < (size_t)m->n_classes * 5; ++blk)
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c) {
                const double v = m->blocks[blk * N * N + (size_t)r * N + c];
                bt[blk * N * N + (size_t)c * N + r] = v;
                b32[blk * N * N + (size_t)c * N + r] = (float)v;
            }
    std::vector<float> c32(m->Ctime.begin(), m->Ctime.end());
    std::vector<int32_t> cls(m->cls.begin(), m->cls.end());
    const int64_t runs = (m->E + 63) / 64;
    std::vector<int32_t> run_cls(runs);
    std::vector<int32_t> mixed;
    for (int64_t r = 0; r < runs; ++r) {
        const int64_t t0 = 64 * r, t1 = std::min<int64_t>(t0 + 64, m->E);
        run_cls[r] = cls[t0];
        for (int64_t e = t0 + 1; e < t1; ++e)
            if (cls[e] != cls[t0]) run_cls[r] = -1;
        if (run_cls[r] < 0)
            for (int64_t e = t0; e < t1; ++e) mixed.push_back((int32_t)e);
    }
    m->d.n_mixed_runs = std::count(run_cls.begin(), run_cls.end(), -1);
    m->d.runs_uniform = m->d.n_mixed_runs == 0 ? 1 : 0;
    m->d.n_mixed_elems = (int64_t)mixed.size();
    STDG_HIP(hipMalloc(&m->d.run_cls, runs * sizeof(int32_t)));
    STDG_HIP(hipMemcpy(m->d.run_cls, run_cls.data(), runs * sizeof(int32_t), hipMemcpyHostToDevice));
    if (!mixed.empty()) {
        STDG_HIP(hipMalloc(&m->d.mixed_elems, mixed.size() * sizeof(int32_t)));
        STDG_HIP(hipMemcpy(m->d.mixed_elems, mixed.data(), mixed.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    STDG_HIP(hipMalloc(&m->d.blocks, nb * sizeof(double)));
    STDG_HIP(hipMalloc(&m->d.blocks32, nb * sizeof(float)));
    STDG_HIP(hipMalloc(&m->d.cls, m->E * sizeof(int32_t)));
    STDG_HIP(hipMalloc(&m->d.nbr, 4 * m->E * sizeof(int32_t)));
    STDG_HIP(hipMalloc(&m->d.C, m->G * m->G * sizeof(double)));
    STDG_HIP(hipMalloc(&m->d.C32, m->G * m->G * sizeof(float)));
    STDG_HIP(hipMemcpy(m->d.blocks, bt.data(), nb * sizeof(double), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d.blocks32, b32.data(), nb * sizeof(float), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d.cls, cls.data(), m->E * sizeof(int32_t), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d.nbr, m->nbr.data(), 4 * m->E * sizeof(int32_t), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d.C, m->Ctime.data(), m->G * m->G * sizeof(double), hipMemcpyHostToDevice));
    STDG_HIP(hipMemcpy(m->d.C32, c32.data(), m->G * m->G * sizeof(float), hipMemcpyHostToDevice));
    {
        const int G = m->G;
        std::vector<real> ci(m->Ctime.begin(), m->Ctime.end());
        lu_inverse(G, ci);
        std::vector<double> cinv(G * G), cid(G * G, 0.0);
        std::vector<float> cinv32(G * G), cid32(G * G, 0.0f);
        for (int i = 0; i < G * G; ++i) { cinv[i] = (double)ci[i]; cinv32[i] = (float)ci[i]; }
        for (int i = 0; i < G; ++i) { cid[i * G + i] = 1.0; cid32[i * G + i] = 1.0f; }
        STDG_HIP(hipMalloc(&m->d.Cinv, G * G * sizeof(double)));
        STDG_HIP(hipMalloc(&m->d.Cinv32, G * G * sizeof(float)));
        STDG_HIP(hipMalloc(&m->d.Cid, G * G * sizeof(double)));
        STDG_HIP(hipMalloc(&m->d.Cid32, G * G * sizeof(float)));
        STDG_HIP(hipMemcpy(m->d.Cinv, cinv.data(), G * G * sizeof(double), hipMemcpyHostToDevice));
        STDG_HIP(hipMemcpy(m->d.Cinv32, cinv32.data(), G * G * sizeof(float), hipMemcpyHostToDevice));
        STDG_HIP(hipMemcpy(m->d.Cid, cid.data(), G * G * sizeof(double), hipMemcpyHostToDevice));
        STDG_HIP(hipMemcpy(m->d.Cid32, cid32.data(), G * G * sizeof(float), hipMemcpyHostToDevice));
    }
    return upload_cg_operands(m);
}

void free_tables(stdg_mesh* m) {
    for (void* p : {(void*)m->d.blocks, (void*)m->d.blocks32, (void*)m->d.aop32, (void*)m->d.cls, (void*)m->d.nbr,
                    (void*)m->d.C, (void*)m->d.C32, (void*)m->d.Cinv, (void*)m->d.Cinv32,
                    (void*)m->d.Cid, (void*)m->d.Cid32, (void*)m->d.chunk_slot, (void*)m->d.chunk_halo,
                    (void*)m->d.lane_ops, (void*)m->d.elem_ops, (void*)m->d.elem_ops64, (void*)m->d.run_cls, (void*)m->d.mixed_elems})
        if (p) (void)hipFree(p);
    m->d = DeviceTables();
}

}  // namespace stdg

using namespace stdg;

extern "C" const char* stdg_last_error(void) { return g_last_error.c_str(); }

static int mesh_build_impl(const double* xyz, int64_t n_vert, const int64_t* tets, int64_t n_tet,
                           const double* nodes, const stdg_config* cfg, stdg_mesh** out, bool device) {
    if (!xyz || !tets || !cfg || !out) { set_error("null argument"); return STDG_ERR_ARG; }
    *out = nullptr;
    if (n_vert < 4 || n_tet < 1 || n_tet > (int64_t)INT32_MAX) { set_error("bad mesh size"); return STDG_ERR_ARG; }
    if (cfg->p < 1 || cfg->p > 6 || cfg->p_gamma < 0 || cfg->p_gamma > 6) {
        set_error("degree out of range (1 <= p <= 6, 0 <= p_gamma <= 6)");
        return STDG_ERR_ARG;
    }
    if (!(cfg->dt > 0.0) || !(cfg->nu >= 0.0)) { set_error("dt must be > 0 and nu >= 0"); return STDG_ERR_ARG; }
    if (cfg->anchor_tet < 0 || cfg->anchor_tet >= n_tet) { set_error("anchor element out of range"); return STDG_ERR_ARG; }
    const int N = (cfg->p + 1) * (cfg->p + 2) * (cfg->p + 3) / 6;
    if (cfg->anchor_node < 0 || cfg->anchor_node >= N) { set_error("anchor node out of range"); return STDG_ERR_ARG; }
    if (cfg->periodic)
        for (int d = 0; d < 3; ++d)
            if (!(cfg->box_hi[d] > cfg->box_lo[d])) { set_error("periodic box is empty"); return STDG_ERR_ARG; }
    stdg_mesh* m = nullptr;
    try {
        m = new stdg_mesh();
        m->cfg = *cfg;
        m->p = cfg->p;
        m->G = cfg->p_gamma + 1;
        m->N = N;
        m->Nst = N * m->G;
        m->E = n_tet;
        std::vector<int64_t> rep;
        int e = build_topology(m, xyz, n_vert, tets, nullptr);
        if (e == STDG_OK && nodes) e = set_geometry(m, nodes);
        if (e == STDG_OK) e = assign_classes(m, rep);
        if (e == STDG_OK && cfg->reorder) {
            const std::vector<int64_t> order = class_chunk_order(m);
            e = build_topology(m, xyz, n_vert, tets, &order);
            if (e == STDG_OK && nodes) e = set_geometry(m, nodes);
            if (e == STDG_OK) e = assign_classes(m, rep);
        }
        if (e == STDG_OK) sort_faces_by_class(m);
        if (e == STDG_OK) e = build_blocks(m, rep);
        // curved elements: the pressure system only (the Picard-step tables
        // assume affine elements)
        if (e == STDG_OK && !m->curved) e = build_picard_tables(m, rep);
        if (e == STDG_OK) {
            m->anchor = m->iperm[cfg->anchor_tet];
            m->anchor_node = cfg->anchor_node;
            if (device) e = upload_tables(m);
            if (device && e == STDG_OK && !m->curved) e = upload_picard_tables(m);
        }
        if (e != STDG_OK) {
            free_picard(m);
            free_tables(m);
            delete m;
            return e;
        }
    } catch (const std::bad_alloc&) {
        if (m) { free_tables(m); delete m; }
        set_error("host allocation failed");
        return STDG_ERR_NOMEM;
    } catch (const std::exception& ex) {
        if (m) { free_tables(m); delete m; }
        set_error(std::string("mesh build failed: ") + ex.what());
        return STDG_ERR_MESH;
    }
    *out = m;
    return STDG_OK;
}

extern "C" int stdg_mesh_build(const double* xyz, int64_t n_vert, const int64_t* tets, int64_t n_tet,
                               const stdg_config* cfg, stdg_mesh** out) {
    return mesh_build_impl(xyz, n_vert, tets, n_tet, nullptr, cfg, out, true);
}

extern "C" int stdg_mesh_build_host(const double* xyz, int64_t n_vert, const int64_t* tets, int64_t n_tet,
                                    const stdg_config* cfg, stdg_mesh** out) {
    return mesh_build_impl(xyz, n_vert, tets, n_tet, nullptr, cfg, out, false);
}

extern "C" int stdg_mesh_build_curved(const double* xyz, int64_t n_vert, const int64_t* tets, int64_t n_tet,
                                      const double* nodes, int32_t host_only, const stdg_config* cfg,
                                      stdg_mesh** out) {
    if (!nodes) { set_error("null argument"); return STDG_ERR_ARG; }
    return mesh_build_impl(xyz, n_vert, tets, n_tet, nodes, cfg, out, host_only == 0);
}

extern "C" int stdg_mesh_blocks(const stdg_mesh* m, double* blocks, int32_t* cls, int32_t* nbr, double* C) {
    if (!m) { set_error("null argument"); return STDG_ERR_ARG; }
    if (blocks) std::memcpy(blocks, m->blocks.data(), m->blocks.size() * sizeof(double));
    if (cls) std::memcpy(cls, m->cls.data(), m->E * sizeof(int32_t));
    if (nbr) std::memcpy(nbr, m->nbr.data(), 4 * m->E * sizeof(int32_t));
    if (C) std::memcpy(C, m->Ctime.data(), m->Ctime.size() * sizeof(double));
    return STDG_OK;
}

extern "C" int stdg_mesh_info_get(const stdg_mesh* m, stdg_mesh_info* info) {
    if (!m || !info) { set_error("null argument"); return STDG_ERR_ARG; }
    info->n_tet = m->E;
    info->n_face = (int64_t)m->faces.size();
    info->n_interior_face = m->n_interior;
    info->N = m->N;
    info->G = m->G;
    info->Nst = m->Nst;
    info->n_classes = m->n_classes;
    info->anchor_internal = m->anchor;
    const bool run = lane_supported(m);
    info->inner_layout = run ? STDG_LAYOUT_RUN : STDG_LAYOUT_ELEMENT;
    info->inner_len = run ? lane_len(m) : m->E * m->G * m->N;
    info->inner_per_element = m->d.elem_ops != nullptr ? 1 : 0;
    return STDG_OK;
}

extern "C" int stdg_mesh_permutation(const stdg_mesh* m, int64_t* perm) {
    if (!m || !perm) { set_error("null argument"); return STDG_ERR_ARG; }
    std::memcpy(perm, m->perm.data(), m->E * sizeof(int64_t));
    return STDG_OK;
}

extern "C" int stdg_mesh_faces(const stdg_mesh* m, int64_t* left, int32_t* lf, int64_t* right, int32_t* rf) {
    if (!m || !left || !lf || !right || !rf) { set_error("null argument"); return STDG_ERR_ARG; }
    for (size_t j = 0; j < m->faces.size(); ++j) {
        left[j] = m->faces[j].left;
        lf[j] = m->faces[j].lf;
        right[j] = m->faces[j].right;
        rf[j] = m->faces[j].rf;
    }
    return STDG_OK;
}

extern "C" void stdg_mesh_free(stdg_mesh* m) {
    if (!m) return;
    free_workspace(m);
    free_picard(m);
    free_tables(m);
    delete m;
}

extern "C" int stdg_pressure_apply(const stdg_mesh* m, int32_t precision, const double* x, double* y,
                                   void* stream) {
    if (!m || !x || !y) { set_error("null argument"); return STDG_ERR_ARG; }
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    if (x == y) { set_error("x and y must not overlap"); return STDG_ERR_ARG; }
    hipStream_t s = (hipStream_t)stream;
    if (precision == STDG_FP64) {
        STDG_HIP(launch_apply_f64(m, x, y, s));
        return STDG_OK;
    }
    if (precision == STDG_FP32) {
        stdg_mesh* mm = const_cast<stdg_mesh*>(m);
        const int64_t n = m->E * m->Nst;
        if (!mm->ws.x32) {
            // scratch FP32 vectors (owned by the handle)
            STDG_HIP(hipMalloc(&mm->ws.x32, n * sizeof(float)));
        }
        if (!mm->ws.q32) STDG_HIP(hipMalloc(&mm->ws.q32, n * sizeof(float)));
        STDG_HIP(convert_d2f(x, mm->ws.x32, n, s));
        STDG_HIP(launch_apply_f32(m, mm->ws.x32, mm->ws.q32, s));
        STDG_HIP(convert_f2d(mm->ws.q32, y, n, s));
        return STDG_OK;
    }
    set_error("unknown precision");
    return STDG_ERR_ARG;
}

extern "C" int stdg_pressure_apply_f32(const stdg_mesh* m, const float* x, float* y, void* stream) {
    if (!m || !x || !y) { set_error("null argument"); return STDG_ERR_ARG; }
    if (!m->d.blocks) { set_error("mesh was built host-only"); return STDG_ERR_ARG; }
    if (x == y) { set_error("x and y must not overlap"); return STDG_ERR_ARG; }
    STDG_HIP(launch_apply_f32(m, x, y, (hipStream_t)stream));
    return STDG_OK;
}

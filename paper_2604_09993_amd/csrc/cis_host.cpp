// Host-only parts of the C ABI: model objects, validation, status text.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "cis_host.hpp"

namespace cis {

static thread_local char g_last_error[512] = "";

cis_status fail(cis_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return st;
}

static bool finite_all(const double* a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

cis_status check_common(const cis_model* m, const cis_shape* sh, const void* X, const void* U,
                        const void* s, const void* params) {
    if (!m || !sh) return fail(CIS_ERR_NULL, "model and shape are required");
    if (sh->dtype != CIS_F64 && sh->dtype != CIS_F32)
        return fail(CIS_ERR_DTYPE, "unknown dtype %d", sh->dtype);
    if (sh->layout < 0 || sh->layout > 4)
        return fail(CIS_ERR_DIM, "cis_shape.layout=%d outside [0, 4]", sh->layout);
    if (sh->N < 1) return fail(CIS_ERR_DIM, "N=%d must be >= 1", sh->N);
    if (sh->substeps < 1 || sh->substeps > 4096)
        return fail(CIS_ERR_DIM, "substeps=%d outside [1, 4096]", sh->substeps);
    if (sh->ld_node < (int64_t)sh->N + 1)
        return fail(CIS_ERR_DIM, "ld_node=%lld < N+1=%d", (long long)sh->ld_node, sh->N + 1);
    if (sh->ld_int < (int64_t)sh->N)
        return fail(CIS_ERR_DIM, "ld_int=%lld < N=%d", (long long)sh->ld_int, sh->N);
    if (!X || !s || !params || (m->m > 0 && !U))
        return fail(CIS_ERR_NULL, "X, s, params (and U when m > 0) are required");
    const size_t es = elem_size(sh->dtype);
    if (!aligned(X, es) || !aligned(U, es) || !aligned(s, es) || !aligned(params, es))
        return fail(CIS_ERR_LAYOUT, "input pointer not aligned to %zu bytes", es);
    return CIS_OK;
}

}  // namespace cis

using cis::fail;
using cis::finite_all;

extern "C" const char* cis_version(void) { return "cis 0.1.0 (gfx950)"; }

extern "C" const char* cis_status_string(cis_status st) {
    switch (st) {
        case CIS_OK: return "ok";
        case CIS_ERR_NULL: return "required pointer is NULL";
        case CIS_ERR_DIM: return "dimension out of range";
        case CIS_ERR_LAYOUT: return "pointer not aligned to the element size";
        case CIS_ERR_DTYPE: return "unsupported dtype";
        case CIS_ERR_WORKSPACE: return "workspace missing or too small";
        case CIS_ERR_MODEL: return "malformed model description";
        case CIS_ERR_HIP: return "HIP runtime error";
        case CIS_ERR_UNSUPPORTED: return "topology has no compiled kernel";
        case CIS_ERR_NONFINITE: return "non-finite values (debug mode)";
    }
    return "unknown status";
}

extern "C" const char* cis_last_error(void) { return cis::g_last_error; }

static bool compiled_topology(int L, int D) {
#define CIS_IS(LL, DD) \
    if (L == LL && D == DD) return true;
    CIS_TOPOLOGIES(CIS_IS)
#undef CIS_IS
    return false;
}

extern "C" cis_status cis_model_create(const cis_model_desc* d, cis_model** out) {
    if (!d || !out) return fail(CIS_ERR_NULL, "cis_model_create: desc and out are required");
    *out = nullptr;
    const int nb = d->n_bodies, nj = d->n_joints, nc = d->n_contacts;
    if (nb < 1 || nj < 0 || nc < 0 || nb > 64 || nj > 64 || nc > 32)
        return fail(CIS_ERR_MODEL, "cis_model_create: counts out of range (nb=%d nj=%d nc=%d)", nb,
                    nj, nc);
    if (!d->link_length) return fail(CIS_ERR_NULL, "cis_model_create: link_length is required");
    if (nj > 0 && (!d->joint_parent || !d->joint_child || !d->joint_anchor_parent ||
                   !d->joint_anchor_child || !d->joint_stiffness || !d->joint_damping))
        return fail(CIS_ERR_NULL, "cis_model_create: joint arrays are required when n_joints > 0");
    if (nc > 0 && (!d->contact_body || !d->contact_point))
        return fail(CIS_ERR_NULL, "cis_model_create: contact arrays are required when n_contacts > 0");
    for (int b = 0; b < nb; ++b)
        if (!(d->link_length[b] > 0.0) || !std::isfinite(d->link_length[b]))
            return fail(CIS_ERR_MODEL, "cis_model_create: link_length[%d] must be finite and > 0", b);
    for (int j = 0; j < nj; ++j)
        if (d->joint_parent[j] < 0 || d->joint_parent[j] >= nb || d->joint_child[j] < 0 ||
            d->joint_child[j] >= nb || d->joint_parent[j] == d->joint_child[j])
            return fail(CIS_ERR_MODEL, "cis_model_create: joint %d has invalid bodies", j);
    for (int i = 0; i < nc; ++i)
        if (d->contact_body[i] < 0 || d->contact_body[i] >= nb)
            return fail(CIS_ERR_MODEL, "cis_model_create: contact %d has an invalid body", i);
    if ((nj && (!finite_all(d->joint_anchor_parent, 2 * nj) ||
                !finite_all(d->joint_anchor_child, 2 * nj) || !finite_all(d->joint_stiffness, nj) ||
                !finite_all(d->joint_damping, nj))) ||
        (nc && !finite_all(d->contact_point, 2 * nc)) || !std::isfinite(d->gravity) ||
        !std::isfinite(d->terrain_amplitude) || !std::isfinite(d->terrain_wavenumber))
        return fail(CIS_ERR_MODEL, "cis_model_create: non-finite model constant");
    // map onto the (legs, depth) family
    int L = nc, D = 0;
    if (L == 0) {
        if (nb != 1 || nj != 0)
            return fail(CIS_ERR_UNSUPPORTED, "cis_model_create: a model without contacts must be one free body");
    } else {
        D = nj / L;
        if (nj != L * D || nb != 1 + L * D)
            return fail(CIS_ERR_UNSUPPORTED, "cis_model_create: not a torso + equal legs topology");
        for (int j = 0; j < nj; ++j) {
            const int parent = (j % D == 0) ? 0 : j;
            if (d->joint_parent[j] != parent || d->joint_child[j] != j + 1)
                return fail(CIS_ERR_UNSUPPORTED, "cis_model_create: joint %d breaks the leg ordering", j);
        }
        for (int i = 0; i < nc; ++i)
            if (d->contact_body[i] != D * (i + 1))
                return fail(CIS_ERR_UNSUPPORTED, "cis_model_create: contact %d is not at a leg tip", i);
    }
    if (!compiled_topology(L, D))
        return fail(CIS_ERR_UNSUPPORTED, "cis_model_create: no kernel compiled for %d legs x %d links", L, D);
    cis_model* m = new cis_model();
    m->nb = nb;
    m->nj = nj;
    m->nc = nc;
    m->L = L;
    m->D = D;
    m->n = 6 * nb;
    m->ny = nc + 1;
    m->nx = m->n + m->ny;
    m->m = 3 * nj + 3 * nc;
    m->np = nb + 2;
    m->len.assign(d->link_length, d->link_length + nb);
    if (nj) {
        m->rp.assign(d->joint_anchor_parent, d->joint_anchor_parent + 2 * nj);
        m->rc.assign(d->joint_anchor_child, d->joint_anchor_child + 2 * nj);
        m->ks.assign(d->joint_stiffness, d->joint_stiffness + nj);
        m->ds.assign(d->joint_damping, d->joint_damping + nj);
    }
    if (nc) m->cr.assign(d->contact_point, d->contact_point + 2 * nc);
    m->g = d->gravity;
    m->A = d->terrain_amplitude;
    m->kappa = d->terrain_wavenumber;
    *out = m;
    return CIS_OK;
}

extern "C" void cis_model_destroy(cis_model* m) { delete m; }

extern "C" cis_status cis_model_dims(const cis_model* m, int32_t* n, int32_t* n_y, int32_t* nu,
                                     int32_t* n_params) {
    if (!m) return fail(CIS_ERR_NULL, "cis_model_dims: model is required");
    if (n) *n = m->n;
    if (n_y) *n_y = m->ny;
    if (nu) *nu = m->m;
    if (n_params) *n_params = m->np;
    return CIS_OK;
}

// Mesh construction: skeleton (Section 2), IMEX partition and interface
// (Section 4), trace map of the element-by-element assembly (eq:assembly),
// stiffness indicator (Section 5), reference operators and device tables.
#include <cmath>
#include <cstring>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "mesh.h"

namespace hfr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

fr_status fail(fr_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

// Gauss-Legendre nodes (ascending) and weights by Newton's method on the
// three-term Legendre recurrence.
static void gauss_legendre(int n, double* x, double* w) {
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (n - i - 0.25) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            double pn = (n == 0) ? 1.0 : p1;
            double pm = (n == 1) ? 1.0 : p0;
            double dp = n * (z * pn - pm) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        double pm = (n == 1) ? 1.0 : p0;
        double dp = n * (z * p1 - pm) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// Gauss-Lobatto-Legendre points: the end points and the roots of the
// derivative of the Legendre polynomial of degree P-1, by Newton's method
// on P'_{P-1} (second derivative from the Legendre equation).
static void gauss_lobatto(int P, double* x) {
    const int n = P - 1;
    x[0] = -1.0;
    x[n] = 1.0;
    for (int i = 1; i < n; ++i) {
        double z = -std::cos(M_PI * i / n);
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            const double pn = (n == 1) ? z : p1, pm = (n == 1) ? 1.0 : p0;
            const double d1 = n * (z * pn - pm) / (z * z - 1.0);
            const double d2 = (2.0 * z * d1 - n * (n + 1.0) * pn) / (1.0 - z * z);
            const double dz = d1 / d2;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        x[i] = z;
    }
}

// Lagrange basis on nodes[0..P) evaluated at t
static double lagrange(const double* nodes, int P, int j, double t) {
    double v = 1.0;
    for (int k = 0; k < P; ++k)
        if (k != j) v *= (t - nodes[k]) / (nodes[j] - nodes[k]);
    return v;
}

RefOps make_ref_ops(int P) {
    RefOps o{};
    o.P = P;
    gauss_legendre(P, o.x, o.w);
    // barycentric weights and the differentiation matrix
    double lam[kMaxP];
    for (int j = 0; j < P; ++j) {
        double prod = 1.0;
        for (int k = 0; k < P; ++k)
            if (k != j) prod *= (o.x[j] - o.x[k]);
        lam[j] = 1.0 / prod;
    }
    for (int i = 0; i < P; ++i) {
        double diag = 0.0;
        for (int j = 0; j < P; ++j) {
            if (i == j) continue;
            double d = (lam[j] / lam[i]) / (o.x[i] - o.x[j]);
            o.D[i * P + j] = d;
            diag -= d;
        }
        o.D[i * P + i] = diag;
    }
    for (int j = 0; j < P; ++j) {
        double a = 1.0, b = 1.0;
        for (int k = 0; k < P; ++k) {
            if (k == j) continue;
            a *= (-1.0 - o.x[k]) / (o.x[j] - o.x[k]);
            b *= (1.0 - o.x[k]) / (o.x[j] - o.x[k]);
        }
        o.lm[j] = a;
        o.lp[j] = b;
        // DG-recovering correction: its divergence at solution point j is
        // the face basis value over the quadrature weight (M^-1 lifting)
        o.cl[j] = a / o.w[j];
        o.cr[j] = b / o.w[j];
    }
    gauss_lobatto(P, o.xg);
    for (int q = 0; q < P; ++q)
        for (int i = 0; i < P; ++i) {
            o.gi[q * P + i] = lagrange(o.xg, P, i, o.x[q]);
            o.gj[i * P + q] = lagrange(o.x, P, q, o.xg[i]);
        }
    return o;
}

}  // namespace hfr

using namespace hfr;

extern "C" const char* fr_last_error(void) {
    return g_last_error.c_str();
}

template <class T>
static fr_status upload(T** dst, const std::vector<T>& src, size_t& bytes) {
    *dst = nullptr;
    if (src.empty()) return FR_OK;
    size_t nb = src.size() * sizeof(T);
    if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess)
        return fail(FR_E_NOMEM, "hipMalloc of mesh table failed");
    if (hipMemcpy(*dst, src.data(), nb, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FR_E_DEVICE, "hipMemcpy of mesh table failed");
    bytes += nb;
    return FR_OK;
}

static void free_mesh_device(fr_mesh_s* m) {
    void* ptrs[] = {m->d_verts, m->d_finfo, m->d_fS, m->d_imp, m->d_exp,
                    m->d_trace_map, m->d_tpside, m->d_efr_fnodes,
                    m->d_efr_inc_ptr, m->d_efr_inc, m->d_dtscale};
    for (void* p : ptrs) (void)hipFree(p);
}

extern "C" fr_status fr_mesh_create(const fr_mesh_desc* d, fr_mesh_t* out) {
    if (!d || !out) return fail(FR_E_INVALID, "null argument");
    *out = nullptr;
    if (d->order < 1 || d->order > FR_MAX_ORDER)
        return fail(FR_E_INVALID, "order out of range");
    if (d->n_elems < 1 || d->n_nodes < 3 || !d->node_xy || !d->elem_nodes)
        return fail(FR_E_INVALID, "empty mesh");
    if (d->physics != FR_PHYS_EULER && d->physics != FR_PHYS_EDAC)
        return fail(FR_E_INVALID, "unknown physics");
    if (d->physics == FR_PHYS_EULER && !(d->gamma > 1.0))
        return fail(FR_E_INVALID, "gamma must be > 1");
    if (d->physics == FR_PHYS_EDAC && !(d->theta > 0.0 && std::isfinite(d->theta)))
        return fail(FR_E_INVALID, "EDAC theta must be positive and finite");
    auto m = new fr_mesh_s();
    const int P = d->order + 1, Ne = d->n_elems;
    m->P = P;
    m->Np = P * P;
    m->Ne = Ne;
    m->ops = make_ref_ops(P);
    m->phys.gamma = d->gamma;
    for (int v = 0; v < 4; ++v) m->phys.uinf[v] = d->uinf[v];
    m->phys.kind = d->physics;
    m->phys.theta = d->theta;
    auto topo = [&](int node) {
        return d->node_topo ? d->node_topo[node] : node;
    };
    for (int e = 0; e < Ne; ++e)
        for (int c = 0; c < 4; ++c) {
            int nd = d->elem_nodes[4 * e + c];
            if (nd < 0 || nd >= d->n_nodes) {
                delete m;
                return fail(FR_E_MESH, "vertex id out of range");
            }
        }
    // ---- skeleton: faces on first encounter ---------------------------
    std::unordered_set<uint64_t> directed;
    std::unordered_map<uint64_t, int> open;
    auto key = [](int64_t a, int64_t b) {
        return (uint64_t(uint32_t(a)) << 32) | uint32_t(b);
    };
    m->elem_face.assign(4 * Ne, -1);
    m->elem_side.assign(4 * Ne, 0);
    for (int e = 0; e < Ne; ++e) {
        for (int lf = 0; lf < 4; ++lf) {
            int a = topo(d->elem_nodes[4 * e + lf]);
            int b = topo(d->elem_nodes[4 * e + (lf + 1) % 4]);
            if (a == b) {
                delete m;
                return fail(FR_E_MESH, "degenerate edge in element " +
                                           std::to_string(e));
            }
            if (!directed.insert(key(a, b)).second) {
                delete m;
                return fail(FR_E_MESH,
                            "edge traversed twice (clockwise or "
                            "non-conforming element " + std::to_string(e) + ")");
            }
            auto it = open.find(key(b, a));
            if (it != open.end()) {
                int f = it->second;
                open.erase(it);
                if (m->face_e[2 * f] == e) {
                    delete m;
                    return fail(FR_E_MESH, "element " + std::to_string(e) +
                                               " is its own neighbour");
                }
                m->face_e[2 * f + 1] = e;
                m->face_l[2 * f + 1] = lf;
                m->elem_face[4 * e + lf] = f;
                m->elem_side[4 * e + lf] = 1;
            } else {
                int f = int(m->face_e.size() / 2);
                m->face_e.push_back(e);
                m->face_e.push_back(-1);
                m->face_l.push_back(lf);
                m->face_l.push_back(-1);
                open[key(a, b)] = f;
                m->elem_face[4 * e + lf] = f;
                m->elem_side[4 * e + lf] = 0;
            }
        }
    }
    const int Nf = int(m->face_e.size() / 2);
    m->Nf = Nf;
    std::vector<int> face_bc(Nf, FR_BC_INTERIOR);
    for (int f = 0; f < Nf; ++f) {
        int e0 = m->face_e[2 * f], l0 = m->face_l[2 * f];
        int tag0 = d->elem_face_bc ? d->elem_face_bc[4 * e0 + l0] : 0;
        if (m->face_e[2 * f + 1] < 0) {
            if (tag0 != FR_BC_WALL && tag0 != FR_BC_FARFIELD) {
                delete m;
                return fail(FR_E_MESH,
                            "unmatched edge without boundary tag (element " +
                                std::to_string(e0) + ", face " +
                                std::to_string(l0) + ")");
            }
            face_bc[f] = tag0;
        } else {
            int e1 = m->face_e[2 * f + 1], l1 = m->face_l[2 * f + 1];
            int tag1 = d->elem_face_bc ? d->elem_face_bc[4 * e1 + l1] : 0;
            if (tag0 || tag1) {
                delete m;
                return fail(FR_E_MESH, "boundary tag on an interior edge");
            }
        }
    }
    // ---- independent instances: no face may join two of them ------------
    if (d->n_instances < 0 || (d->n_instances > 0 && !d->elem_instance)) {
        delete m;
        return fail(FR_E_INVALID, "n_instances needs elem_instance");
    }
    if (d->n_instances > 0) {
        m->n_instances = d->n_instances;
        m->instance.assign(d->elem_instance, d->elem_instance + Ne);
        for (int e = 0; e < Ne; ++e)
            if (m->instance[e] < 0 || m->instance[e] >= d->n_instances) {
                delete m;
                return fail(FR_E_INVALID, "elem_instance out of range");
            }
        for (int f = 0; f < Nf; ++f) {
            const int e0 = m->face_e[2 * f], e1 = m->face_e[2 * f + 1];
            if (e1 >= 0 && m->instance[e0] != m->instance[e1]) {
                delete m;
                return fail(FR_E_MESH, "a face joins elements of two instances (face " +
                                           std::to_string(f) + ")");
            }
        }
    }
    // ---- geometry, validity and stiffness indicator --------------------
    m->verts.resize(8 * size_t(Ne));
    m->es.resize(Ne);
    for (int e = 0; e < Ne; ++e) {
        double xc[4], yc[4];
        for (int c = 0; c < 4; ++c) {
            int nd = d->elem_nodes[4 * e + c];
            xc[c] = d->node_xy[2 * nd];
            yc[c] = d->node_xy[2 * nd + 1];
            m->verts[8 * e + c] = xc[c];
            m->verts[8 * e + 4 + c] = yc[c];
        }
        // bilinear Jacobian is linear in each variable: positive at the
        // four corners <=> positive everywhere
        for (int c = 0; c < 4; ++c) {
            double xi = (c == 1 || c == 2) ? 1.0 : -1.0;
            double et = (c >= 2) ? 1.0 : -1.0;
            double x_xi = 0.25 * ((xc[1] - xc[0]) * (1 - et) + (xc[2] - xc[3]) * (1 + et));
            double y_xi = 0.25 * ((yc[1] - yc[0]) * (1 - et) + (yc[2] - yc[3]) * (1 + et));
            double x_et = 0.25 * ((xc[3] - xc[0]) * (1 - xi) + (xc[2] - xc[1]) * (1 + xi));
            double y_et = 0.25 * ((yc[3] - yc[0]) * (1 - xi) + (yc[2] - yc[1]) * (1 + xi));
            if (!(x_xi * y_et - x_et * y_xi > 0.0)) {
                delete m;
                return fail(FR_E_MESH, "non-positive Jacobian (clockwise or "
                                       "folded) in element " + std::to_string(e));
            }
        }
        double area = 0.0, per = 0.0;
        for (int c = 0; c < 4; ++c) {
            int c1 = (c + 1) % 4;
            area += xc[c] * yc[c1] - xc[c1] * yc[c];
            per += std::hypot(xc[c1] - xc[c], yc[c1] - yc[c]);
        }
        m->es[e] = 0.5 * area / per;
    }
    // ---- partition ------------------------------------------------------
    std::vector<char> mask(Ne);
    for (int e = 0; e < Ne; ++e)
        mask[e] = d->implicit_mask ? (d->implicit_mask[e] != 0)
                                   : (m->es[e] <= d->es_cutoff);
    m->elem_to_imp.assign(Ne, -1);
    for (int e = 0; e < Ne; ++e) {
        if (mask[e]) {
            m->elem_to_imp[e] = int(m->imp.size());
            m->imp.push_back(e);
        } else {
            m->exp.push_back(e);
        }
    }
    m->Nim = int(m->imp.size());
    m->Nex = int(m->exp.size());
    m->face_kind.resize(Nf);
    m->trace_of_face.assign(Nf, -1);
    for (int f = 0; f < Nf; ++f) {
        int e0 = m->face_e[2 * f], e1 = m->face_e[2 * f + 1];
        int k;
        if (e1 < 0) k = FR_FACE_BOUNDARY;
        else if (mask[e0] && mask[e1]) k = FR_FACE_TRACE;
        else if (mask[e0] || mask[e1]) k = FR_FACE_UPSILON;
        else k = FR_FACE_EXPLICIT;
        m->face_kind[f] = k;
        if (k == FR_FACE_TRACE) {
            m->trace_of_face[f] = int(m->trace_faces.size());
            m->trace_faces.push_back(f);
        }
        if (k == FR_FACE_UPSILON) m->n_upsilon++;
        if (k == FR_FACE_BOUNDARY) m->n_boundary++;
    }
    m->Ntf = int(m->trace_faces.size());
    m->Ntp = m->Ntf * P;
    m->efr = (d->flags & FR_MESH_EFR) != 0;
    if (m->efr) {
        // nodes over the trace faces in order, owner counter-clockwise:
        // start vertex (if new), interior GLL nodes, end vertex (if new)
        std::unordered_map<int, int> vnode;
        m->efr_fnodes.assign(size_t(m->Ntf) * P, -1);
        int nn = 0;
        for (int F = 0; F < m->Ntf; ++F) {
            const int f = m->trace_faces[F];
            const int e0 = m->face_e[2 * f], l0 = m->face_l[2 * f];
            const int va = topo(d->elem_nodes[4 * e0 + l0]);
            const int vb = topo(d->elem_nodes[4 * e0 + (l0 + 1) % 4]);
            auto ia = vnode.find(va);
            if (ia == vnode.end()) ia = vnode.emplace(va, nn++).first;
            m->efr_fnodes[size_t(F) * P] = ia->second;
            for (int i = 1; i < P - 1; ++i) m->efr_fnodes[size_t(F) * P + i] = nn++;
            auto ib = vnode.find(vb);
            if (ib == vnode.end()) ib = vnode.emplace(vb, nn++).first;
            m->efr_fnodes[size_t(F) * P + P - 1] = ib->second;
        }
        m->Ntp = nn;
    }
    m->trace_map.assign(size_t(m->Nim) * 4 * P, -1);
    std::vector<int> tpside(m->efr ? 0 : 2 * size_t(m->Ntp), -1);
    for (int k = 0; k < m->Nim && m->efr; ++k) {
        int e = m->imp[k];
        for (int lf = 0; lf < 4; ++lf) {
            int tf = m->trace_of_face[m->elem_face[4 * e + lf]];
            if (tf < 0) continue;
            int side = m->elem_side[4 * e + lf];
            for (int i = 0; i < P; ++i)
                m->trace_map[(size_t(k) * 4 + lf) * P + i] =
                    m->efr_fnodes[size_t(tf) * P + (side ? P - 1 - i : i)];
        }
    }
    if (m->efr) {
        // incidences of every node: slots (imp*4+lf)*P+i in slot order
        m->efr_inc_ptr.assign(size_t(m->Ntp) + 1, 0);
        for (size_t s = 0; s < m->trace_map.size(); ++s)
            if (m->trace_map[s] >= 0) m->efr_inc_ptr[m->trace_map[s] + 1]++;
        for (int a = 0; a < m->Ntp; ++a) m->efr_inc_ptr[a + 1] += m->efr_inc_ptr[a];
        m->efr_inc.assign(m->efr_inc_ptr[m->Ntp], -1);
        std::vector<int> fill(m->efr_inc_ptr.begin(), m->efr_inc_ptr.end() - 1);
        for (size_t s = 0; s < m->trace_map.size(); ++s)
            if (m->trace_map[s] >= 0) m->efr_inc[fill[m->trace_map[s]]++] = int(s);
    }
    for (int k = 0; k < m->Nim && !m->efr; ++k) {
        int e = m->imp[k];
        for (int lf = 0; lf < 4; ++lf) {
            int f = m->elem_face[4 * e + lf];
            int tf = m->trace_of_face[f];
            if (tf < 0) continue;
            int side = m->elem_side[4 * e + lf];
            for (int q = 0; q < P; ++q) {
                int tp = tf * P + (side ? P - 1 - q : q);
                m->trace_map[(size_t(k) * 4 + lf) * P + q] = tp;
                tpside[2 * size_t(tp) + side] = (k * 4 + lf) * P + q;
            }
        }
    }
    // ---- per element-face flux roles and face-owned normals -------------
    m->finfo.resize(4 * size_t(Ne));
    m->fS.resize(8 * size_t(Ne));
    for (int e = 0; e < Ne; ++e) {
        for (int lf = 0; lf < 4; ++lf) {
            int f = m->elem_face[4 * e + lf];
            int side = m->elem_side[4 * e + lf];
            FaceInfo fi{};
            fi.nb_e = m->face_e[2 * f + 1 - side];
            fi.nb_lf = m->face_l[2 * f + 1 - side];
            fi.trace = -1;
            int k = m->face_kind[f];
            if (k == FR_FACE_BOUNDARY) {
                const bool wall = face_bc[f] == FR_BC_WALL;
                if (m->elem_to_imp[e] >= 0)
                    fi.role = wall ? ROLE_WALL_T : ROLE_FAR_T;
                else
                    fi.role = wall ? ROLE_WALL : ROLE_FAR;
            }
            else if (k == FR_FACE_TRACE) {
                fi.role = ROLE_HFR;
                fi.trace = m->trace_of_face[f] * 2 + side;
            } else
                fi.role = ROLE_RUSANOV;
            if (fi.nb_e < 0) {
                fi.nb_e = e;
                fi.nb_lf = lf;
            }
            m->finfo[4 * e + lf] = fi;
            // scaled outward normal J_f n of a straight edge, constant
            // along it: the owner's edge vector rotated, halved; the
            // neighbour uses its negation so both sides share one value
            int eo = m->face_e[2 * f], lo = m->face_l[2 * f];
            const double* vx = &m->verts[8 * eo];
            const double* vy = vx + 4;
            int a = lo, b = (lo + 1) % 4;
            double sx = 0.5 * (vy[b] - vy[a]);
            double sy = -0.5 * (vx[b] - vx[a]);
            if (side) {
                sx = -sx;
                sy = -sy;
            }
            m->fS[8 * e + 2 * lf] = sx;
            m->fS[8 * e + 2 * lf + 1] = sy;
        }
    }
    // ---- device tables ---------------------------------------------------
    m->host_only = (d->flags & FR_MESH_HOST_ONLY) != 0;
    if (m->host_only) {
        *out = m;
        return FR_OK;
    }
    fr_status st;
    size_t& nb = m->device_bytes;
    if ((st = upload(&m->d_verts, m->verts, nb)) ||
        (st = upload(&m->d_finfo, m->finfo, nb)) ||
        (st = upload(reinterpret_cast<double**>(&m->d_fS), m->fS, nb)) ||
        (st = upload(&m->d_imp, m->imp, nb)) ||
        (st = upload(&m->d_exp, m->exp, nb)) ||
        (st = upload(&m->d_trace_map, m->trace_map, nb)) ||
        (!m->efr && (st = upload(&m->d_tpside, tpside, nb))) ||
        (m->efr && (st = upload(&m->d_efr_fnodes, m->efr_fnodes, nb))) ||
        (m->efr && (st = upload(&m->d_efr_inc_ptr, m->efr_inc_ptr, nb))) ||
        (m->efr && (st = upload(&m->d_efr_inc, m->efr_inc, nb))) ||
        (m->n_instances > 0 &&
         (st = upload(&m->d_dtscale, std::vector<double>(Ne, 1.0), nb)))) {
        free_mesh_device(m);
        delete m;
        return st;
    }
    *out = m;
    return FR_OK;
}

extern "C" fr_status fr_mesh_set_instance_dt(fr_mesh_t m, const double* dt) {
    if (!m || !dt) return fail(FR_E_INVALID, "null argument");
    if (m->n_instances == 0) return fail(FR_E_INVALID, "mesh has no instances");
    if (m->host_only) return fail(FR_E_INVALID, "host-only mesh");
    for (int i = 0; i < m->n_instances; ++i)
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i]))
            return fail(FR_E_INVALID, "instance time steps must be positive and finite");
    std::vector<double> sc(m->Ne);
    for (int e = 0; e < m->Ne; ++e) sc[e] = dt[m->instance[e]];
    if (hipMemcpy(m->d_dtscale, sc.data(), sizeof(double) * sc.size(),
                  hipMemcpyHostToDevice) != hipSuccess)
        return fail(FR_E_DEVICE, "upload of instance time steps failed");
    return FR_OK;
}

extern "C" void fr_mesh_destroy(fr_mesh_t m) {
    if (!m) return;
    free_mesh_device(m);
    delete m;
}

extern "C" fr_status fr_mesh_get_info(fr_mesh_t m, fr_mesh_info* o) {
    if (!m || !o) return fail(FR_E_INVALID, "null argument");
    o->order = m->P - 1;
    o->n_pts = m->Np;
    o->n_elems = m->Ne;
    o->n_faces = m->Nf;
    o->n_implicit = m->Nim;
    o->n_explicit = m->Nex;
    o->n_trace_faces = m->Ntf;
    o->n_trace_points = m->Ntp;
    o->n_upsilon = m->n_upsilon;
    o->n_boundary = m->n_boundary;
    o->n_loc = 4 * m->Np;
    o->m_loc = 16 * m->P;
    o->device_table_bytes = m->device_bytes;
    o->efr = m->efr ? 1 : 0;
    o->n_instances = m->n_instances;
    return FR_OK;
}

extern "C" fr_status fr_mesh_get_maps(fr_mesh_t m, int32_t* face_elem,
                                      int32_t* face_local, int32_t* face_kind,
                                      int32_t* trace_map,
                                      int32_t* implicit_elems,
                                      int32_t* explicit_elems, double* es,
                                      double* sol_xy) {
    if (!m) return fail(FR_E_INVALID, "null mesh");
    if (face_elem) std::memcpy(face_elem, m->face_e.data(), 8 * size_t(m->Nf));
    if (face_local) std::memcpy(face_local, m->face_l.data(), 8 * size_t(m->Nf));
    if (face_kind) std::memcpy(face_kind, m->face_kind.data(), 4 * size_t(m->Nf));
    if (trace_map && !m->trace_map.empty())
        std::memcpy(trace_map, m->trace_map.data(), 4 * m->trace_map.size());
    if (implicit_elems && m->Nim)
        std::memcpy(implicit_elems, m->imp.data(), 4 * size_t(m->Nim));
    if (explicit_elems && m->Nex)
        std::memcpy(explicit_elems, m->exp.data(), 4 * size_t(m->Nex));
    if (es) std::memcpy(es, m->es.data(), 8 * size_t(m->Ne));
    if (sol_xy) {
        const int P = m->P;
        for (int e = 0; e < m->Ne; ++e) {
            const double* vx = &m->verts[8 * e];
            const double* vy = vx + 4;
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    double xi = m->ops.x[i], et = m->ops.x[j];
                    double N0 = 0.25 * (1 - xi) * (1 - et), N1 = 0.25 * (1 + xi) * (1 - et);
                    double N2 = 0.25 * (1 + xi) * (1 + et), N3 = 0.25 * (1 - xi) * (1 + et);
                    size_t o = (size_t(e) * m->Np + j * P + i) * 2;
                    sol_xy[o] = N0 * vx[0] + N1 * vx[1] + N2 * vx[2] + N3 * vx[3];
                    sol_xy[o + 1] = N0 * vy[0] + N1 * vy[1] + N2 * vy[2] + N3 * vy[3];
                }
        }
    }
    return FR_OK;
}

extern "C" fr_status fr_explicit_rhs(fr_mesh_t m, const double* u, double* R,
                                     void* stream) {
    if (!m || !u || (!R && m->Nex)) return fail(FR_E_INVALID, "null argument");
    if (m->host_only) return fail(FR_E_INVALID, "host-only mesh");
    if (m->Nex == 0) return FR_OK;
    ResidualLaunch a{};
    a.list = m->d_exp;
    a.nlist = m->Nex;
    a.u = u;
    a.Ne = m->Ne;
    a.verts = m->d_verts;
    a.finfo = m->d_finfo;
    a.fS = m->d_fS;
    a.uhat = nullptr;
    a.phys = m->phys;
    a.R = R;
    HIP_TRY(launch_residual(m->ops, a, hipStream_t(stream)));
    return FR_OK;
}

extern "C" fr_status fr_modal_filter(fr_mesh_t m, const fr_filter_params* prm,
                                     double* u, void* stream) {
    if (!m || !prm || !u) return fail(FR_E_INVALID, "null argument");
    if (m->host_only) return fail(FR_E_INVALID, "host-only mesh");
    const double alpha = prm->alpha, sx = prm->s, ec = prm->eta_c, kap = prm->kappa;
    if (!std::isfinite(alpha) || !std::isfinite(sx) || !std::isfinite(ec) ||
        !std::isfinite(kap) || alpha < 0.0 || sx <= 0.0 || kap < 0.0)
        return fail(FR_E_INVALID, "filter parameters: need alpha >= 0, s > 0, "
                                  "kappa >= 0, all finite");
    FilterLaunch f{};
    f.P = m->P;
    for (int q = 0; q < m->P; ++q) {
        const double x = m->ops.x[q];
        f.w[q] = m->ops.w[q];
        double p0 = 1.0, p1 = x;          // Legendre three-term recurrence
        for (int a = 0; a < m->P; ++a) {
            double pa = a == 0 ? 1.0 : x;
            if (a >= 2) {
                pa = ((2 * a - 1) * x * p1 - (a - 1) * p0) / a;
                p0 = p1;
                p1 = pa;
            }
            f.v1[q * m->P + a] = std::sqrt(a + 0.5) * pa;
        }
    }
    const int emax = 2 * (m->P - 1);   // exponent sum of the top mode
    for (int e = 0; e <= emax; ++e) {
        double sg = 1.0;
        if (e >= ec && emax > ec)
            sg = std::exp(-alpha * std::pow((e - ec) / (emax - ec), sx));
        f.sig[e] = std::pow(sg, kap);
    }
    HIP_TRY(launch_modal_filter(f, 4L * m->Ne, u, hipStream_t(stream)));
    return FR_OK;
}

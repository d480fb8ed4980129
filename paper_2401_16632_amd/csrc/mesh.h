// Host-side mesh object (opaque to ABI callers).
#pragma once

#include <vector>

#include "internal.h"

struct fr_mesh_s {
    int P = 0, Np = 0, Ne = 0, Nf = 0, Nim = 0, Nex = 0, Ntf = 0, Ntp = 0;
    int n_upsilon = 0, n_boundary = 0;
    hfr::RefOps ops{};
    hfr::Physics phys{};
    // host tables
    std::vector<int> face_e, face_l;      // [Nf][2]
    std::vector<int> face_kind;           // [Nf]
    std::vector<int> elem_face, elem_side;// [Ne][4]
    std::vector<int> imp, exp, elem_to_imp;
    std::vector<int> trace_of_face;       // [Nf], -1 off trace
    std::vector<int> trace_faces;         // [Ntf] face id
    std::vector<int> trace_map;           // [Nim][4][P]
    std::vector<double> es;               // [Ne]
    std::vector<double> verts;            // [Ne][8]
    std::vector<hfr::FaceInfo> finfo;     // [Ne][4]
    std::vector<double> fS;               // [Ne][4][2]
    // device tables
    double* d_verts = nullptr;
    hfr::FaceInfo* d_finfo = nullptr;
    double2* d_fS = nullptr;
    int* d_imp = nullptr;
    int* d_exp = nullptr;
    int* d_trace_map = nullptr;           // [Nim][4][P]
    int* d_tpside = nullptr;              // [Ntp][2]: (imp*4+lf)*P+q_el
    size_t device_bytes = 0;
    bool host_only = false;
    // interior-embedded trace (FR_MESH_EFR): Ntp counts trace nodes
    bool efr = false;
    std::vector<int> efr_fnodes;          // [Ntf][P] nodes, owner ccw order
    std::vector<int> efr_inc_ptr;         // [Ntp+1] node -> incidences
    std::vector<int> efr_inc;             // slot (imp*4+lf)*P+i, element ccw i
    int* d_efr_fnodes = nullptr;
    int* d_efr_inc_ptr = nullptr;
    int* d_efr_inc = nullptr;
    // independent instances: element -> instance, and the per-element
    // factor of every time step (the instance's dt), 1 until set
    int n_instances = 0;
    std::vector<int> instance;            // [Ne]
    double* d_dtscale = nullptr;          // [Ne] or null (all 1)
};

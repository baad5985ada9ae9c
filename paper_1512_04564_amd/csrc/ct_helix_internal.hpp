// Internal declarations of the 3-D helical part (not part of the public ABI).
#pragma once

#include <vector>

#include "../../include/ct_helix.h"
#include "ct_helix_body.hpp"
#include "ct_internal.hpp"

namespace ct {

// Host tables of a helical scan (FP64 geometry stored FP32), before upload.
struct HelixTables {
    GeomTables fan;              // transaxial fan-beam tables of every view (bnd, scale, inv, rowsweep)
    std::vector<float2> cs;      // [nviews] (cos b, sin b)
    std::vector<float> zai, zaf; // [nviews] (S_z - z_lo) / dz: integer part, fraction in [0, 1)
    std::vector<float> wr;       // [nr + 1] w_r / (dsd dz)
    std::vector<float> secphi;   // [nr][nb]
    float dwn = 0.f;             // dw / (dsd dz)
};

// The transaxial descriptor of a helical scan: its views as a multi-turn fan beam.
ct_geom_desc helix_fan_desc(const ct_helix_desc &d);
ct_status check_helix_desc(const ct_helix_desc *d);
ct_status helix_tables(const ct_helix_desc &d, HelixTables &t);

}  // namespace ct

// cg_capi_internal.hpp -- host helpers shared by the context API and the
// serving engine: parameter validation, buffer layout, descriptor filling and
// launch planning.
#pragma once

#include <string>

#include "cg_device.hpp"
#include "cglbm.h"

struct lbm_ctx;

namespace cgi {

struct Layout {
    int elem = 4;            // bytes per stored population
    int pitch = 0;           // row pitch in elements (multiple of 64)
    long long plane = 0;     // elements per plane
    size_t buf_bytes = 0;    // one buffer: 18 planes
};

int fail(lbm_ctx *c, int code, const std::string &msg);
int validate(const lbm_params *p, std::string &msg);
Layout layout(const lbm_params *p);
void fill_desc(const lbm_params *p, cgd::SlotDesc &d);
int default_tx(int nx, int ny);
int plan_strip(int nx, int ny, int tx, int req);
void set_geometry(cgd::SlotDesc &d, const lbm_params *p, const Layout &L, int tx, int strip);

}  // namespace cgi

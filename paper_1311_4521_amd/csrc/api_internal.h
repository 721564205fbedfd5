// Functions of the C-ABI implementation shared between its source files
// (internal to libtmhop).
#pragma once

#include <stddef.h>

#include "../../include/tmhop.h"

namespace tmh_api {

// Argument checks of tmh_qtm_apply (null pointers, sign, precision, aliasing).
tmh_status qtm_check(const tmh_lattice* l, const void* out, const void* gauge, const void* in, double kappa,
                     double mu, const double theta[4], int sign, tmh_prec prec);
// Qhat(sign) in -> out through the even field te (tmh_spinor_bytes(l, prec)
// bytes), enqueued on the handle's stream; with timed = false no timing
// events are recorded (none created).  The device of l must be current.
tmh_status qtm_run(tmh_lattice* l, void* out, const void* gauge, const void* in, void* te, double kappa,
                   double mu, const double theta[4], int sign, tmh_prec prec, bool timed);
int lattice_device(const tmh_lattice* l);
size_t lattice_spinor_bytes(const tmh_lattice* l, tmh_prec prec);

// Fixed device scratch of the allocation-free entry points (noalloc.hip):
// queries and keeps the address of the current device's copy, which must
// be `device`.
tmh_status noalloc_setup(int device);

}  // namespace tmh_api

// Entry points declared in iga_trim.h whose kernels are not in this build yet.
#include "plan.hpp"

extern "C" {
int iga_trim_mass_form_batched(iga_plan* const*, int32_t, const iga_coeff*, double* const*, int32_t, void*) {
    iga::set_error("batched formation not built");
    return IGA_E_UNSUPPORTED;
}
}

#pragma once
#include <stddef.h>
#include <stdint.h>

#include "pm.h"

namespace pm {
int fit_model(const pm_counts *P, const double *T, size_t m, uint32_t proj,
              pm_model *out, double *cond, double *resid, uint32_t *rank);
}

// Single translation unit of libapmg: the kernels and the C ABI.
#include <algorithm>
#include <cstring>
#include <type_traits>

#include "../../include/apmg.h"
#include "apmg_device.h"
#include "apmg_kernels.h"

#include "apmg_mlp.hip"
#include "apmg_adjoint.hip"
#include "apmg_misc.hip"
#include "apmg_sort.hip"
#include "apmg_dd.hip"
#include "apmg_scatter.hip"
#include "apmg_variants.hip"
#include "apmg_abi.hip"

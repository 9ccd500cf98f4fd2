"""MI355X-native k-blocked LR-CCSD sigma path (HIP for gfx950).

The compute path is the C-ABI library liblrcc.so (include/lrcc.h); this
package is only its Python binding (argument marshalling, no arithmetic).
"""
from .lrcc import Context, Group, LrccError, lib, measure_peaks, plan_check, FP64, FP32  # noqa: F401

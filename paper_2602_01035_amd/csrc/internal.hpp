// Host-side checks shared by the fusion entry points and the serving loop (not exported).
#pragma once
#include "fuseflow.h"

namespace ff {

// Everything about one frame, its parameters and its output that the host can check
// before any launch: parameter ranges, camera range, non-null images and output arrays,
// colour on every view when colour is asked for.  FF_OK or FF_ERR_INVALID_ARG.
ff_status check_frame(const ff_frame& fr, const ff_params& prm, const ff_output& out);

// Copy every per-shape tuning of src into dst (contexts of one process).
void share_tuning(const ff_context* src, ff_context* dst);

}  // namespace ff

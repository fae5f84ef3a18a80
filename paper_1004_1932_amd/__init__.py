"""MI355X (gfx950) library for the all-pairs Oseen step of active spring
dumbbell suspensions (Putz, Dunkel, Yeomans, "CUDA simulations of active
dumbbell suspensions"). The compute path is libad.so (include/ad.h); this
package holds its sources, its build script, a thin ctypes binding and the
host-side observables of the paper's pair and array experiments."""
from .binding import (  # noqa: F401
    ADError, Simulator, ad_create, ad_destroy, ad_workspace_size, ad_bind_workspace, ad_set_launch,
    ad_get_launch, ad_set_state, ad_get_state, ad_forces, ad_mobility_apply, ad_step, ad_run, ad_check,
    ad_use_graph, ad_profile_pairs, ad_profile_read, ad_last_error, make_params, lib, LIB_PATH,
    ad_sa_rhs, ad_sa_workspace_size, ad_sa_run, StrokeAveraged, ad_mobility_apply_static, ad_valu_probe,
)
from . import observables  # noqa: F401

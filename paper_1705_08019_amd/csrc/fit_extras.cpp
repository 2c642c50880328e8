// Optional per-handle workspaces (adjoint state) are released here.
#include "fit_host.hpp"

namespace fit {
void grid_release_extras(fit_grid* g) { (void)g; }
}  // namespace fit

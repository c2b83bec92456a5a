"""MI355X (gfx950) clotting-step library: one segregated finite-volume time step of the
clotFoam model (PISO with a Brinkman term, eta, ADP release, TVD transport with reactive
injury walls, RK4 reactions) behind a C ABI (include/clot.h)."""

"""FD-preconditioned flexible GMRES for spline collocation systems on MI355X (gfx950)."""

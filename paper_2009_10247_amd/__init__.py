"""MI355X (gfx950) engine for linear-algebraic T_P fixpoints over sparse program matrices."""

"""MI355X (gfx950) 2-D CDF 5/3 DWT with the non-separable lifting scheme."""

// Analytical cost model (filled in below).

"""MI355X-native fused HLBM stream-collide (homogenized hybrid recursive-
regularized LBM with Smagorinsky LES and a Spalding wall model for moving
porous rotors) behind a C-ABI library of hand-written gfx950 HIP kernels."""

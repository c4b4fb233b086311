"""MI355X-native Gaussian-process profile-likelihood engine (gfx950, HIP)."""

"""MI355X-native upwind-DG convection (binding to the HIP library; filled in below)."""

"""MI355X-native EnVar forward-ensemble engine (batched MAC-grid Navier-Stokes + anomaly gradient)."""

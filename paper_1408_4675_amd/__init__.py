"""MI355X-native k-space pseudospectral solver (Jaros, Rendell & Treeby,
nonlinear ultrasound on distributed clusters, Section 2.2)."""

"""VSA-OGM hot path on MI355X (gfx950): encode, bundle, decode, classify behind a C ABI."""

"""MI355X-native fast bilateral stereo (placeholder; filled in with the binding)."""
